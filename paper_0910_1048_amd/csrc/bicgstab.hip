// Multishift BiCGStab for the shifted systems of the Neuberger rational function
// (the BiCGStab variant named beside BiCG-LR in the section "Two-sided Lanczos
// with rational functions"); only H_W is applied, never its adjoint.
//
// Systems (A' - sigma_i) x_i = y, A' = c^2 H_W(mu)^2, y = c H_W (I - P) b.  Seed:
// the shift of smallest modulus, M = A' - sigma_seed, shadow r^ = y:
//   v = M p,  alpha = r^^H r / r^^H v,  s = r - alpha v,  t = M s,
//   omega = t^H s / t^H t,  r' = s - omega t,
//   beta = (alpha / omega) r^^H r' / r^^H r,  p' = r' + beta (p - omega v).
// alpha and beta are BiCG's, so the BiCG factors zeta_i carry over; the
// stabilising polynomial of shift i (M + tau_i, tau_i = sigma_seed - sigma_i)
// uses omega_i = omega / (1 + omega tau_i) and adds the factor pi_i = prod (1 +
// omega tau_i).  With r_i = zeta_i r / pi_i and s_i = zeta_i' s / pi_i:
//   x_i += alpha_i p_i + omega_i s_i,
//   p_i' = r_i' + beta_i (p_i - (omega_i / alpha_i)(r_i - s_i)),
// alpha_i = alpha zeta_i' / zeta_i, beta_i = beta (zeta_i' / zeta_i)^2; every shift's
// p_i and x_i are kept (one pass over all of them per iteration).  FP64; the
// scalars are formed on the host from deterministic block partial sums, three
// synchronisations per iteration.
#include <chrono>
#include <complex>
#include <vector>

#include "field_io.h"
#include "vec.h"

namespace sgn {

namespace {

using zc = std::complex<double>;
constexpr int kBsShifts = SGN_MAX_POLES;

__device__ __forceinline__ z64 ld(const double2 *p, int64_t e)
{
    const double2 v = p[e];
    return {v.x, v.y};
}
__device__ __forceinline__ void st(double2 *p, int64_t e, z64 v) { p[e] = make_double2(v.r, v.i); }

// s = r - alpha v
__global__ void __launch_bounds__(256) bs_sub_kernel(const double2 *r, const double2 *v, z64 alpha, double2 *s,
                                                     int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        st(s, e, ld(r, e) - alpha * ld(v, e));
}

// partials: t^H s and t^H t per block
__global__ void __launch_bounds__(256) bs_dots_kernel(const double2 *t, const double2 *s, int64_t n, z64 *part)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 tv = ld(t, e), sv = ld(s, e);
        const z64 d = cmulc(tv, sv);
        a += d.r;
        b += d.i;
        c += norm2(tv);
    }
    __shared__ double lds[12];
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = {v[0], v[1]};
        part[2 * blockIdx.x + 1] = {v[2], 0.0};
    }
}

// r' = s - omega t; partials r^^H r' and ||r'||^2
__global__ void __launch_bounds__(256) bs_res_kernel(const double2 *s, const double2 *t, z64 omega, const double2 *rh,
                                                     double2 *r, int64_t n, z64 *part)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 rv = ld(s, e) - omega * ld(t, e);
        st(r, e, rv);
        const z64 d = cmulc(ld(rh, e), rv);
        a += d.r;
        b += d.i;
        c += norm2(rv);
    }
    __shared__ double lds[12];
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = {v[0], v[1]};
        part[2 * blockIdx.x + 1] = {v[2], 0.0};
    }
}

// Per active shift i (coefficients cf[6 i .. 6 i + 5] = a, b, c, d, e, f):
//   x_i += a p_i + b s;   p_i = c r' + d p_i + e r + f s
struct BsShift {
    int idx;
    int pad;
};
__global__ void __launch_bounds__(256) bs_shift_kernel(const double2 *rn, const double2 *ro, const double2 *s,
                                                       double2 *P, double2 *X, int64_t n, int na, const BsShift *act,
                                                       const z64 *cf)
{
    __shared__ z64 c[6 * kBsShifts];
    __shared__ int id[kBsShifts];
    for (int k = threadIdx.x; k < 6 * na; k += blockDim.x) c[k] = cf[k];
    for (int k = threadIdx.x; k < na; k += blockDim.x) id[k] = act[k].idx;
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 rv = ld(rn, e), rov = ld(ro, e), sv = ld(s, e);
        for (int k = 0; k < na; ++k) {
            double2 *Pi = P + (int64_t)id[k] * n;
            double2 *Xi = X + (int64_t)id[k] * n;
            const z64 *q = c + 6 * k;
            const z64 p = ld(Pi, e);
            st(Xi, e, ld(Xi, e) + q[0] * p + q[1] * sv);
            st(Pi, e, q[2] * rv + q[3] * p + q[4] * rov + q[5] * sv);
        }
    }
}

// x = sum_i w_i X_i
__global__ void __launch_bounds__(256) bs_combine_kernel(const double2 *X, const double *w, int ns, int64_t n,
                                                         double2 *x)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        z64 acc = {0.0, 0.0};
        for (int i = 0; i < ns; ++i) acc = acc + w[i] * ld(X + (int64_t)i * n, e);
        st(x, e, acc);
    }
}

template <typename T> __global__ void bs_fill_kernel(T *p, T v, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

struct DeviceScratch {
    void *p = nullptr;
    explicit DeviceScratch(size_t bytes)
    {
        if (bytes && hipMalloc(&p, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "bicgstab scratch"};
    }
    ~DeviceScratch()
    {
        if (p) (void)hipFree(p);
    }
};

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// sums of nb blocks of 2 partials each (fixed order): {sum of part[2b], sum of part[2b+1]}
void host_sums(const z64 *dpart, int nb, hipStream_t s, zc &a, zc &b)
{
    std::vector<z64> h(2 * (size_t)nb);
    SGN_HIP(hipMemcpyAsync(h.data(), dpart, sizeof(z64) * 2 * nb, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    a = b = 0.0;
    for (int k = 0; k < nb; ++k) {
        a += zc(h[2 * k].r, h[2 * k].i);
        b += zc(h[2 * k + 1].r, h[2 * k + 1].i);
    }
}

zc host_sum1(const z64 *dpart, int nb, hipStream_t s)
{
    std::vector<z64> h(nb);
    SGN_HIP(hipMemcpyAsync(h.data(), dpart, sizeof(z64) * nb, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    zc a = 0.0;
    for (int k = 0; k < nb; ++k) a += zc(h[k].r, h[k].i);
    return a;
}

sgn_status solve_one(const sgn_problem &pb, const sgn_rational &rf, const sgn_ms_opts &o, sgn_stats *stp,
                     hipStream_t s)
{
    const auto t_start = std::chrono::steady_clock::now();
    SGN_REQUIRE(pb.lat && pb.b && pb.x, "multishift_bicgstab: null problem field");
    SGN_REQUIRE(std::isfinite(pb.mu), "multishift_bicgstab: mu not finite");
    Lattice &lat = *as_lattice(pb.lat);
    Context &ctx = *lat.ctx;
    SGN_HIP(hipSetDevice(ctx.device));
    const int ns = rf.s;
    const int64_t n = 12 * lat.S, nc = 12 * lat.V;
    const size_t b64 = (size_t)n * 16, c64 = (size_t)nc * 16;
    sgn_stats st{};
    st.nshift = ns;
    // workspace: r, ro, rh, v, sv, t, tmp, x, canonical staging, P_i and X_i of every shift, coefficients
    const size_t cbytes = sizeof(z64) * 6 * kBsShifts + sizeof(BsShift) * kBsShifts + sizeof(double) * kBsShifts;
    char *a = static_cast<char *>(ctx.ensure_arena(8 * b64 + c64 + 2 * (size_t)ns * b64 + cbytes));
    double2 *r = reinterpret_cast<double2 *>(a), *ro = r + n, *rh = ro + n, *v = rh + n, *sv = v + n, *t = sv + n,
            *tmp = t + n, *xi = tmp + n;
    char *rcan = reinterpret_cast<char *>(xi + n);
    double2 *P = reinterpret_cast<double2 *>(rcan + c64), *X = P + (size_t)ns * n;
    z64 *dcf = reinterpret_cast<z64 *>(X + (size_t)ns * n);
    BsShift *dact = reinterpret_cast<BsShift *>(dcf + 6 * kBsShifts);
    double *dw = reinterpret_cast<double *>(dact + kBsShifts);
    const int nvb = vec_blocks(n);
    const int nbs = std::max(dslash_blocks(lat), 2 * nvb);
    z64 *part = static_cast<z64 *>(ctx.ensure_partials(sizeof(z64) * nbs));

    int seed = 0;
    for (int i = 1; i < ns; ++i)
        if (std::abs(rf.sigma[i]) < std::abs(rf.sigma[seed])) seed = i;
    const double s0 = rf.sigma[seed], c2 = rf.c * rf.c;
    OpSpec op;
    op.mu = pb.mu;
    // x = x_P, y = c H (I - P) b
    deflation_prologue(ctx, pb.defl, nc, pb.b, pb.x, rcan, nullptr, s);
    pack_spinor(lat, rcan, tmp, SGN_PREC_F64, s);
    {
        Epilogue ep;
        ep.a = rf.c;
        dslash_launch(lat, SGN_PREC_F64, op, tmp, r, ep, s);
    }
    const double ynorm = norm_sync(ctx, r, n, false, s);
    SGN_REQUIRE(std::isfinite(ynorm), "multishift_bicgstab: b contains NaN or Inf");
    if (ynorm == 0.0) {
        SGN_HIP(hipStreamSynchronize(s));
        if (stp) *stp = st;
        return SGN_OK;
    }
    SGN_HIP(hipMemcpyAsync(rh, r, b64, hipMemcpyDeviceToDevice, s));
    for (int i = 0; i < ns; ++i) SGN_HIP(hipMemcpyAsync(P + (size_t)i * n, r, b64, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(bs_fill_kernel<double2>, dim3(nvb), dim3(256), 0, s, X, make_double2(0.0, 0.0), (int64_t)ns * n);
    SGN_HIP(hipGetLastError());
    std::vector<zc> zeta(ns, 1.0), zeta_prev(ns, 1.0), zeta_next(ns), pi(ns, 1.0), pi_next(ns);
    std::vector<double> tau(ns);
    for (int i = 0; i < ns; ++i) tau[i] = s0 - rf.sigma[i];
    std::vector<char> active(ns, 1);
    zc alpha_prev = 1.0, beta_prev = 0.0, rho = zc(ynorm * ynorm, 0.0);
    double rnorm = ynorm;
    const double lim = o.tol * ynorm;
    const int maxiter = o.maxiter > 0 ? o.maxiter : 10000;
    int it = 0;
    bool converged = false, breakdown = false;
    std::vector<z64> cf(6 * (size_t)ns);
    std::vector<BsShift> act;
    const auto t_kry = std::chrono::steady_clock::now();
    while (it < maxiter) {
        double2 *p = P + (size_t)seed * n;
        // v = M p (partials of r^^H v)
        dslash_launch(lat, SGN_PREC_F64, op, p, tmp, Epilogue{}, s);
        Epilogue ep;
        ep.a = c2;
        ep.z = p;
        ep.b = {-s0, 0.0};
        ep.w = rh;
        ep.partials = part;
        const int nb1 = dslash_launch(lat, SGN_PREC_F64, op, tmp, v, ep, s);
        const zc den = host_sum1(part, nb1, s);
        if (!(std::abs(den) > 0.0) || !(std::abs(rho) > 0.0)) {
            breakdown = true;
            break;
        }
        const zc alpha = rho / den;
        for (int i = 0; i < ns; ++i) {
            zeta_next[i] = zeta[i];
            if (!active[i]) continue;
            const zc z = zeta[i], zp = zeta_prev[i];
            const zc dn = alpha_prev * (1.0 + tau[i] * alpha) * zp + alpha * beta_prev * (zp - z);
            zeta_next[i] = z * zp * alpha_prev / dn;
        }
        // s = r - alpha v;  t = M s;  t^H s, t^H t
        hipLaunchKernelGGL(bs_sub_kernel, dim3(nvb), dim3(256), 0, s, r, v, z64{alpha.real(), alpha.imag()}, sv, n);
        dslash_launch(lat, SGN_PREC_F64, op, sv, tmp, Epilogue{}, s);
        Epilogue et;
        et.a = c2;
        et.z = sv;
        et.b = {-s0, 0.0};
        dslash_launch(lat, SGN_PREC_F64, op, tmp, t, et, s);
        hipLaunchKernelGGL(bs_dots_kernel, dim3(nvb), dim3(256), 0, s, t, sv, n, part);
        SGN_HIP(hipGetLastError());
        zc ts, tt;
        host_sums(part, nvb, s, ts, tt);
        const zc om = tt.real() > 0.0 ? ts / tt : zc(0.0, 0.0);
        // r' = s - omega t (the old r kept for the shift updates)
        std::swap(r, ro);
        hipLaunchKernelGGL(bs_res_kernel, dim3(nvb), dim3(256), 0, s, sv, t, z64{om.real(), om.imag()}, rh, r, n,
                           part);
        SGN_HIP(hipGetLastError());
        zc rho_new, rr;
        host_sums(part, nvb, s, rho_new, rr);
        rnorm = std::sqrt(rr.real());
        const bool om_zero = om == zc(0.0, 0.0);
        const zc beta = om_zero ? zc(0.0, 0.0) : (alpha / om) * (rho_new / rho);
        // shift updates
        act.clear();
        for (int i = 0; i < ns; ++i) {
            pi_next[i] = pi[i];
            if (!active[i]) continue;
            const zc ai = alpha * zeta_next[i] / zeta[i];
            const zc q = zeta_next[i] / zeta[i];
            const zc bi = beta * q * q;
            const zc oi = om / (1.0 + om * tau[i]);
            pi_next[i] = pi[i] * (1.0 + om * tau[i]);
            const zc cr = zeta[i] / pi[i], cs = zeta_next[i] / pi[i];
            const zc k = (std::abs(ai) > 0.0) ? bi * oi / ai : zc(0.0, 0.0);
            const zc c6[6] = {ai, oi * cs, zeta_next[i] / pi_next[i], bi, -k * cr, k * cs};
            const size_t j = act.size();
            for (int u = 0; u < 6; ++u) cf[6 * j + u] = {c6[u].real(), c6[u].imag()};
            act.push_back(BsShift{i, 0});
        }
        SGN_HIP(hipMemcpyAsync(dcf, cf.data(), sizeof(z64) * 6 * act.size(), hipMemcpyHostToDevice, s));
        SGN_HIP(hipMemcpyAsync(dact, act.data(), sizeof(BsShift) * act.size(), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(bs_shift_kernel, dim3(nvb), dim3(256), 0, s, r, ro, sv, P, X, n, (int)act.size(), dact, dcf);
        SGN_HIP(hipGetLastError());
        SGN_HIP(hipStreamSynchronize(s));  // the coefficient buffers are rewritten next iteration
        zeta_prev = zeta;
        zeta = zeta_next;
        pi = pi_next;
        alpha_prev = alpha;
        beta_prev = beta;
        rho = rho_new;
        ++it;
        bool all = true;
        for (int i = 0; i < ns; ++i) {
            const double ri = std::abs(zeta[i] / pi[i]) * rnorm;
            st.shift_residual[i] = ri / ynorm;
            if (active[i] && ri <= lim) active[i] = 0;
            if (active[i]) all = false;
        }
        if (all) {
            converged = true;
            break;
        }
        active[seed] = 1;  // the seed drives the recurrence
        if (!std::isfinite(rnorm)) {
            breakdown = true;
            break;
        }
        if (om_zero) break;  // s was already the solution direction: stagnation
    }
    // x = x_P + sum_i omega_i x_i
    SGN_HIP(hipMemcpyAsync(dw, rf.omega, sizeof(double) * ns, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(bs_combine_kernel, dim3(nvb), dim3(256), 0, s, X, dw, ns, n, xi);
    SGN_HIP(hipGetLastError());
    unpack_spinor(lat, xi, rcan, SGN_PREC_F64, s);
    if (pb.defl && pb.defl->m > 0) {  // the exact x_i lie in range(I - P): drop rounding components
        DeviceScratch cd(sizeof(z64) * pb.defl->m);
        deflate_dots(pb.defl->L, pb.defl->m, rcan, nc, static_cast<z64 *>(cd.p), ctx, s);
        deflate_combine(rcan, {1.0, 0.0}, {-1.0, 0.0}, pb.defl->R, pb.defl->m, static_cast<const z64 *>(cd.p),
                        nullptr, nc, s);
        SGN_HIP(hipStreamSynchronize(s));
    }
    axpby64({1.0, 0.0}, rcan, {1.0, 0.0}, pb.x, nc, s);
    if (pb.x_shift)
        for (int i = 0; i < ns; ++i)
            if (pb.x_shift[i]) unpack_spinor(lat, X + (size_t)i * n, pb.x_shift[i], SGN_PREC_F64, s);
    SGN_HIP(hipStreamSynchronize(s));
    st.iterations = it;
    st.matvecs = 4 * it + 1;
    double mx = 0.0;
    for (int i = 0; i < ns; ++i) mx = std::max(mx, st.shift_residual[i]);
    st.residual = mx;
    st.krylov_ms = ms_since(t_kry);
    st.total_ms = ms_since(t_start);
    if (stp) *stp = st;
    if (breakdown) return SGN_ERR_BREAKDOWN;
    return converged ? SGN_OK : SGN_ERR_NOT_CONVERGED;
}

}  // namespace

}  // namespace sgn

using namespace sgn;

extern "C" sgn_status multishift_bicgstab(const sgn_problem *pb, int nprob, const sgn_rational *rf,
                                          const sgn_ms_opts *o, sgn_stats *st, void *stream)
{
    sgn_status result = SGN_OK;
    sgn_status g = guard([&] {
        SGN_REQUIRE(pb && rf && o && nprob >= 0, "multishift_bicgstab: null argument");
        SGN_REQUIRE(rf->s >= 1 && rf->s <= SGN_MAX_POLES && rf->c > 0, "multishift_bicgstab: bad rational function");
        SGN_REQUIRE(o->tol > 0 && o->tol < 1, "multishift_bicgstab: tol must be in (0, 1)");
        SGN_REQUIRE(o->prec == SGN_PREC_F64, "multishift_bicgstab: FP64 only");
        for (int k = 0; k < nprob; ++k) {
            const sgn_status sk = solve_one(pb[k], *rf, *o, st ? st + k : nullptr, static_cast<hipStream_t>(stream));
            if (sk != SGN_OK && result == SGN_OK) result = sk;
        }
    });
    return g != SGN_OK ? g : result;
}
