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
// alpha_i = alpha zeta_i' / zeta_i, beta_i = beta (zeta_i' / zeta_i)^2.
//
// Two forms of the same iteration:
//  * stored basis (default): the seed's r_k and s_k are kept in slots, the seed
//    keeps p and x, and the non-seed p_i, x_i are linear combinations of the
//    slots whose coefficients follow from the recorded alpha, omega, beta; the
//    omega-weighted sum of the non-seed solutions is one lift at the end.  All
//    scalars stay on the device (one-block kernels), the iterations between two
//    host polls are captured once as a HIP graph, and the mixed schedule of the
//    BiCG solver applies (FP64 while the seed residual is above theta32, then
//    FP32 vectors and stencil, FP16 links below theta16, FP64 reliable updates
//    of the seed);
//    When the x_i are requested each is one more lift at the end;
//  * per-shift vectors (basis_slots < 0): FP64, every shift's p_i and x_i updated
//    each iteration, scalars formed on the host from deterministic block partial
//    sums, three synchronisations per iteration.
#include <chrono>
#include <map>
#include <memory>
#include <complex>
#include <vector>

#include "field_io.h"
#include "launch.h"
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

sgn_status solve_explicit(const sgn_problem &pb, const sgn_rational &rf, const sgn_ms_opts &o, sgn_stats *stp,
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

double shift_residual64(Lattice &lat, const OpSpec &op, double c2, double sigma, const void *y, const void *x,
                        void *out, void *tmp, hipStream_t s)
{
    dslash_launch(lat, SGN_PREC_F64, op, x, tmp, Epilogue{}, s);
    Epilogue ep;
    ep.a = -c2;
    ep.z = x;
    ep.b = {sigma, 0.0};
    dslash_launch(lat, SGN_PREC_F64, op, tmp, out, ep, s);
    const int64_t n = 12 * lat.S;
    axpby64({1.0, 0.0}, y, {1.0, 0.0}, out, n, s);
    return norm_sync(*lat.ctx, out, n, false, s);
}

int refine_shift64(Lattice &lat, const OpSpec &op, double c2, double sigma, void *r, void *x, double target,
                   int maxiter, void *work, void *tmp, hipStream_t s, int *matvecs)
{
    Context &ctx = *lat.ctx;
    const int64_t n = 12 * lat.S;
    const size_t b = (size_t)n * 16;
    char *w = static_cast<char *>(work);
    void *rh = w, *pv = w + b, *v = w + 2 * b, *sv = w + 3 * b, *t = w + 4 * b, *e = w + 5 * b;
    auto applyM = [&](const void *in, void *out) {
        dslash_launch(lat, SGN_PREC_F64, op, in, tmp, Epilogue{}, s);
        Epilogue ep;
        ep.a = c2;
        ep.z = in;
        ep.b = {-sigma, 0.0};
        dslash_launch(lat, SGN_PREC_F64, op, tmp, out, ep, s);
        *matvecs += 2;
    };
    auto dot = [&](const void *a, const void *bb) {
        const z64 d = dot_sync(ctx, a, bb, n, false, s);
        return zc(d.r, d.i);
    };
    auto zz = [](zc a) { return z64{a.real(), a.imag()}; };
    SGN_HIP(hipMemcpyAsync(rh, r, b, hipMemcpyDeviceToDevice, s));
    SGN_HIP(hipMemcpyAsync(pv, r, b, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(bs_fill_kernel<double2>, dim3(vec_blocks(n)), dim3(256), 0, s, (double2 *)e,
                       make_double2(0.0, 0.0), n);
    SGN_HIP(hipGetLastError());
    zc rho = dot(rh, r);
    int it = 0;
    while (it < maxiter) {
        applyM(pv, v);
        const zc den = dot(rh, v);
        if (std::abs(den) == 0.0 || std::abs(rho) == 0.0) break;
        const zc alpha = rho / den;
        SGN_HIP(hipMemcpyAsync(sv, r, b, hipMemcpyDeviceToDevice, s));
        axpby64(zz(-alpha), v, {1.0, 0.0}, sv, n, s);  // s = r - alpha v
        applyM(sv, t);
        const double tt = norm_sync(ctx, t, n, false, s);
        const zc omega = tt > 0.0 ? dot(t, sv) / (tt * tt) : zc(0.0);
        axpby64(zz(alpha), pv, {1.0, 0.0}, e, n, s);
        axpby64(zz(omega), sv, {1.0, 0.0}, e, n, s);
        SGN_HIP(hipMemcpyAsync(r, sv, b, hipMemcpyDeviceToDevice, s));
        axpby64(zz(-omega), t, {1.0, 0.0}, r, n, s);  // r = s - omega t
        ++it;
        if (norm_sync(ctx, r, n, false, s) <= target || omega == zc(0.0)) break;
        const zc rho_new = dot(rh, r);
        const zc beta = (rho_new / rho) * (alpha / omega);
        rho = rho_new;
        axpby64(zz(-omega), v, {1.0, 0.0}, pv, n, s);  // p = r + beta (p - omega v)
        axpby64({1.0, 0.0}, r, zz(beta), pv, n, s);
    }
    axpby64({1.0, 0.0}, e, {1.0, 0.0}, x, n, s);
    return it;
}

namespace {

// ----------------------------------------------------------------------------- stored-basis form
struct BsHead {
    z64 rho, alpha, omega, beta, alpha_prev, beta_prev;
    double rnorm, rmax, ynorm, tol, delta, theta32, theta16;
    int iter, maxiter, done, breakdown, reliable, want_phase, phase, ns, seed, go;
};
struct BsState {
    BsHead h;
    z64 zeta[kBsShifts], zeta_prev[kBsShifts], zeta_next[kBsShifts], pi[kBsShifts];
    double tau[kBsShifts];
    int act[kBsShifts];
};
// scalars of iteration k: alpha_k, omega_k, beta_k and ||r_{k+1}||
struct BsHist {
    z64 alpha, omega, beta;
    double rnorm, pad;
};

__device__ __forceinline__ z64 bs_div(z64 a, z64 b)
{
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
__device__ __forceinline__ bool bs_finite(z64 a) { return isfinite(a.r) && isfinite(a.i); }

template <typename R> struct BsVec;
template <> struct BsVec<double> { using t = double2; };
template <> struct BsVec<float> { using t = float2; };
// the slot pointers come from device-side tables: state the global address space
template <typename T> __device__ __forceinline__ z64 ldz(const T *p, int64_t e)
{
    const T v = ((const SGN_GLOBAL T *)p)[e];
    return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stz(double2 *p, int64_t e, z64 v)
{
    ((SGN_GLOBAL double2 *)p)[e] = make_double2(v.r, v.i);
}
__device__ __forceinline__ void stz(float2 *p, int64_t e, z64 v)
{
    ((SGN_GLOBAL float2 *)p)[e] = make_float2((float)v.r, (float)v.i);
}
// Non-temporal forms, for data that the iteration touches once or for the last time: the seed's
// FP64 x (read and written once per iteration), the stored s_k slots (read again only by the
// final lift), t in the r' update and s, v in the x, p update.  They keep such streams from
// evicting the links and the vectors the next kernels read.
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ z64 ldz_nt(const double2 *p, int64_t e)
{
    const nt_d2 v = __builtin_nontemporal_load((const SGN_GLOBAL nt_d2 *)p + e);
    return {v.x, v.y};
}
__device__ __forceinline__ z64 ldz_nt(const float2 *p, int64_t e)
{
    const nt_f2 v = __builtin_nontemporal_load((const SGN_GLOBAL nt_f2 *)p + e);
    return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stz_nt(double2 *p, int64_t e, z64 v)
{
    __builtin_nontemporal_store(nt_d2{v.r, v.i}, (SGN_GLOBAL nt_d2 *)p + e);
}
__device__ __forceinline__ void stz_nt(float2 *p, int64_t e, z64 v)
{
    __builtin_nontemporal_store(nt_f2{(float)v.r, (float)v.i}, (SGN_GLOBAL nt_f2 *)p + e);
}

// alpha = rho / r^^H v from the dotting stencil's partials; the BiCG factors zeta_next
// The one-block scalar steps are bound by memory latency: each issues all its loads (the flags,
// the partials and, in the thread of each shift, that shift's state) before the first use.
static_assert(kBsShifts <= 256, "one thread per shift in the 256-thread scalar kernels");

__device__ __forceinline__ void bs_alpha_kernel_body(BsState *S, const z64 *part, int nb)
{
    const int done = S->h.done, ns = S->h.ns, i = threadIdx.x;
    const z64 rho = S->h.rho, ap = S->h.alpha_prev, bp = S->h.beta_prev;
    double re = 0.0, im = 0.0;
    for (int b = i; b < nb; b += blockDim.x) {
        re += part[b].r;
        im += part[b].i;
    }
    int act = 0;
    z64 z = {0.0, 0.0}, zp = {0.0, 0.0};
    double tau = 0.0;
    if (i < ns) {
        act = S->act[i];
        z = S->zeta[i];
        zp = S->zeta_prev[i];
        tau = S->tau[i];
    }
    if (done) return;
    __shared__ double lds[8];
    __shared__ int bad;
    __shared__ z64 al_sh;
    double v[2] = {re, im};
    block_sum<2>(v, lds);
    if (i == 0) {
        const z64 den = {v[0], v[1]};
        z64 a = bs_div(rho, den);
        bad = 0;
        if (!(den.r * den.r + den.i * den.i > 0.0) || !bs_finite(a)) {
            S->h.breakdown = 1;
            S->h.done = 1;
            a = {0.0, 0.0};
            bad = 1;
        }
        S->h.alpha = a;
        al_sh = a;
    }
    __syncthreads();
    if (bad || i >= ns) return;
    if (!act) {
        S->zeta_next[i] = z;
        return;
    }
    const z64 al = al_sh;
    const z64 one_tau = {1.0 + tau * al.r, tau * al.i};
    S->zeta_next[i] = bs_div(z * zp * ap, ap * one_tau * zp + al * bp * (zp - z));
}
__global__ void __launch_bounds__(256) bs_alpha_kernel(BsState *S, const z64 *part, int nb)
{
    bs_alpha_kernel_body(S, part, nb);
}

// s = r_k - alpha v (r_k read from its slot), into the work vector and the slot of iteration k
template <typename R>
__device__ __forceinline__ void bs_sub_stored_body(const BsState *S, void *const *rslots, const typename BsVec<R>::t *v,
                              typename BsVec<R>::t *s, void *const *sslots, int64_t n)
{
    using T = typename BsVec<R>::t;
    if (S->h.done) return;
    const z64 al = S->h.alpha;
    const T *r = static_cast<const T *>(rslots[S->h.iter]);
    T *slot = static_cast<T *>(sslots[S->h.iter]);
    // r_k is next read by the lift, v only after two stencils: non-temporal reads keep them from
    // displacing the links in the Infinity Cache before the stencil that follows
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 sv = ldz_nt(r, e) - al * ldz_nt(v, e);
        stz(s, e, sv);
        stz_nt(slot, e, sv);
    }
}
template <typename R>
__global__ void __launch_bounds__(256) bs_sub_stored(const BsState *S, void *const *rslots, const typename BsVec<R>::t *v,
                              typename BsVec<R>::t *s, void *const *sslots, int64_t n)
{
    bs_sub_stored_body<R>(S, rslots, v, s, sslots, n);
}

// omega = t^H s / t^H t (0 when t = 0: s was the exact residual 0), from the partials
// {s^H t, ||t||^2} per block of the stencil that produced t
__device__ __forceinline__ void bs_omega_kernel_body(BsState *S, const z64 *part, int nb)
{
    const int done = S->h.done;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        a += part[2 * i].r;
        b += part[2 * i].i;
        c += part[2 * i + 1].r;
    }
    if (done) return;
    __shared__ double lds[12];
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) S->h.omega = v[2] > 0.0 ? z64{v[0] / v[2], -v[1] / v[2]} : z64{0.0, 0.0};
}
__global__ void __launch_bounds__(256) bs_omega_kernel(BsState *S, const z64 *part, int nb)
{
    bs_omega_kernel_body(S, part, nb);
}

// r' = s - omega t into the slot of iteration k + 1 (the residual lives only there);
// partials of r^^H r' and ||r'||^2 (of the stored values)
template <typename R>
__device__ __forceinline__ void bs_res_stored_body(const BsState *S, const typename BsVec<R>::t *s, const typename BsVec<R>::t *t,
                              const typename BsVec<R>::t *rh, void *const *rslots, int64_t n, z64 *part)
{
    using T = typename BsVec<R>::t;
    if (S->h.done) return;
    const z64 om = S->h.omega;
    T *r = static_cast<T *>(rslots[S->h.iter + 1]);
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        z64 rv = ldz(s, e) - om * ldz_nt(t, e);
        if constexpr (sizeof(R) == 4) rv = {(double)(float)rv.r, (double)(float)rv.i};  // as stored
        stz(r, e, rv);
        const z64 d = cmulc(ldz(rh, e), rv);
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
template <typename R>
__global__ void __launch_bounds__(256) bs_res_stored(const BsState *S, const typename BsVec<R>::t *s, const typename BsVec<R>::t *t,
                              const typename BsVec<R>::t *rh, void *const *rslots, int64_t n, z64 *part)
{
    bs_res_stored_body<R>(S, s, t, rh, rslots, n, part);
}

// beta, the history entry, the shifted residual estimates and the control flags
__device__ __forceinline__ void bs_beta_kernel_body(BsState *S, const z64 *part, int nb, BsHist *hist, int cap)
{
    const int done = S->h.done, ns = S->h.ns, i = threadIdx.x;
    const z64 om = S->h.omega;
    const double lim = S->h.tol * S->h.ynorm;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int bk = i; bk < nb; bk += blockDim.x) {
        a += part[2 * bk].r;
        b += part[2 * bk].i;
        c += part[2 * bk + 1].r;
    }
    int act = 0;
    z64 z = {0.0, 0.0}, zn = {0.0, 0.0}, pi = {0.0, 0.0};
    double tau = 0.0;
    if (i < ns) {
        act = S->act[i];
        z = S->zeta[i];
        zn = S->zeta_next[i];
        pi = S->pi[i];
        tau = S->tau[i];
    }
    if (done) {
        if (i == 0) S->h.go = 0;
        return;
    }
    __shared__ double lds[12];
    __shared__ int any, bad;
    __shared__ double rn_sh;
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        const z64 rho_new = {v[0], v[1]};
        const double rn = sqrt(v[2]);
        const z64 al = S->h.alpha;
        const bool om0 = om.r == 0.0 && om.i == 0.0;
        z64 be = om0 ? z64{0.0, 0.0} : bs_div(al, om) * bs_div(rho_new, S->h.rho);
        bad = 0;
        if (!bs_finite(be) || !isfinite(rn) || (!om0 && !(norm2(S->h.rho) > 0.0))) {
            S->h.breakdown = 1;
            S->h.done = 1;
            be = {0.0, 0.0};
            bad = 1;
        }
        const int k = S->h.iter;
        if (k < cap) hist[k] = BsHist{al, om, be, rn, 0.0};
        S->h.go = bad ? 0 : 1;
        S->h.beta = be;
        S->h.rho = rho_new;
        S->h.rnorm = rn;
        S->h.rmax = fmax(S->h.rmax, rn);
        S->h.alpha_prev = al;
        S->h.beta_prev = be;
        S->h.iter = k + 1;
        if (S->h.phase >= 1 && rn < S->h.delta * S->h.rmax) S->h.reliable = 1;
        if (S->h.phase == 0 && rn < S->h.theta32 * S->h.ynorm) S->h.want_phase = 1;
        if (S->h.phase == 1 && rn < S->h.theta16 * S->h.ynorm) S->h.want_phase = 2;
        if (om0) S->h.done = 1;  // t = 0: s, and so r', is zero
        rn_sh = rn;
        any = 0;
    }
    __syncthreads();
    if (bad) return;
    const double rn = rn_sh;
    if (i < ns && act) {
        S->zeta_prev[i] = z;
        S->zeta[i] = zn;
        const z64 f = {1.0 + om.r * tau, om.i * tau};
        const z64 pn = pi * f;
        S->pi[i] = pn;
        const double ri = sqrt(norm2(zn) / norm2(pn)) * rn;
        if (ri <= lim) {
            S->act[i] = 0;
        } else {
            atomicOr(&any, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!any) S->h.done = 1;
        S->act[S->h.seed] = 1;  // the seed drives the recurrence
        if (S->h.iter >= S->h.maxiter) S->h.done = 1;
    }
}
__global__ void __launch_bounds__(256) bs_beta_kernel(BsState *S, const z64 *part, int nb, BsHist *hist, int cap)
{
    bs_beta_kernel_body(S, part, nb, hist, cap);
}

// the seed: x += alpha p + omega s (x in FP64), p = r' + beta (p - omega v), r' read from its
// slot (the iteration counter was advanced by the beta step)
__device__ __forceinline__ void bs_xp64_body(const BsState *S, double2 *p, const double2 *v, void *const *rslots, const double2 *s,
                              double2 *x, int64_t n)
{
    if (!S->h.go || S->h.breakdown) return;
    const z64 al = S->h.alpha, om = S->h.omega, be = S->h.beta;
    const double2 *r = static_cast<const double2 *>(rslots[S->h.iter]);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 pv = ldz(p, e), sv = ldz_nt(s, e);
        stz_nt(x, e, ldz_nt(x, e) + al * pv + om * sv);
        stz(p, e, ldz(r, e) + be * (pv - om * ldz_nt(v, e)));
    }
}
__global__ void __launch_bounds__(256) bs_xp64(const BsState *S, double2 *p, const double2 *v, void *const *rslots, const double2 *s,
                              double2 *x, int64_t n)
{
    bs_xp64_body(S, p, v, rslots, s, x, n);
}

// FP32 phase: p, v, r', s in the [6][S] float4 layout (chunk c holds components 2c, 2c+1), x in
// FP64 [12][S].  An FP32 increment of x (folded into an FP64 base at each reliable update) would
// save a third of this kernel's bytes, but a reliable update hands the seed's true residual to
// every shifted system through the collinear residuals, so the increment's rounding becomes an
// error of the non-seed solutions: at 24^3 x 48 the unverified result moved from 1.4e-9 to
// 7.6e-9 of the verified one.
__device__ __forceinline__ void bs_xp32_body(const BsState *S, float4 *p, const float4 *v, void *const *rslots, const float4 *s,
                              double2 *x, int Sst)
{
    if (!S->h.go || S->h.breakdown) return;
    const z64 al = S->h.alpha, om = S->h.omega, be = S->h.beta;
    const float4 *r = static_cast<const float4 *>(rslots[S->h.iter]);
    const int64_t np = (int64_t)6 * Sst;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < np; f += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(f / Sst), st = (int)(f - (int64_t)c2 * Sst);
        const float4 p4 = p[f], r4 = r[f];
        const nt_f4 s4 = __builtin_nontemporal_load((const SGN_GLOBAL nt_f4 *)s + f);
        const nt_f4 v4 = __builtin_nontemporal_load((const SGN_GLOBAL nt_f4 *)v + f);
        const z64 p0 = {p4.x, p4.y}, p1 = {p4.z, p4.w}, s0 = {s4.x, s4.y}, s1 = {s4.z, s4.w};
        const int64_t e0 = (int64_t)(2 * c2) * Sst + st, e1 = e0 + Sst;
        stz_nt(x, e0, ldz_nt(x, e0) + al * p0 + om * s0);
        stz_nt(x, e1, ldz_nt(x, e1) + al * p1 + om * s1);
        const z64 q0 = z64{r4.x, r4.y} + be * (p0 - om * z64{v4.x, v4.y});
        const z64 q1 = z64{r4.z, r4.w} + be * (p1 - om * z64{v4.z, v4.w});
        p[f] = make_float4((float)q0.r, (float)q0.i, (float)q1.r, (float)q1.i);
    }
}
__global__ void __launch_bounds__(256) bs_xp32(const BsState *S, float4 *p, const float4 *v, void *const *rslots, const float4 *s,
                              double2 *x, int Sst)
{
    bs_xp32_body(S, p, v, rslots, s, x, Sst);
}

// out (+)= sum_j coef_j slot_j (FP64 or FP32 slots; out in the FP64 layout)
constexpr int kBsLiftChunk = 256;
struct BsSlot {
    const void *p;
    int f32;
    int pad;
};
__global__ void __launch_bounds__(256) bs_lift_kernel(const BsSlot *slots, const z64 *coef, int K, int Sst,
                                                      double2 *out)
{
    __shared__ BsSlot sl[kBsLiftChunk];
    __shared__ z64 cf[kBsLiftChunk];
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        sl[j] = slots[j];
        cf[j] = coef[j];
    }
    __syncthreads();
    const int64_t np = (int64_t)6 * Sst;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < np; f += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(f / Sst), st = (int)(f - (int64_t)c2 * Sst);
        const int64_t e0 = (int64_t)(2 * c2) * Sst + st, e1 = e0 + Sst;
        z64 a0 = ldz(out, e0), a1 = ldz(out, e1);
        for (int j = 0; j < K; ++j) {
            const z64 c = cf[j];
            if (c.r == 0.0 && c.i == 0.0) continue;  // uniform
            z64 v0, v1;
            if (sl[j].f32) {
                const float4 t = static_cast<const float4 *>(sl[j].p)[f];
                v0 = {(double)t.x, (double)t.y};
                v1 = {(double)t.z, (double)t.w};
            } else {
                const double2 *q = static_cast<const double2 *>(sl[j].p);
                v0 = ldz(q, e0);
                v1 = ldz(q, e1);
            }
            a0 = a0 + c * v0;
            a1 = a1 + c * v1;
        }
        stz(out, e0, a0);
        stz(out, e1, a1);
    }
}

// Several lifts in one pass over the slots: outs[o] (o < nout <= kLiftOut) = sum_j coef[j kLiftOut + o]
// slot_j (+ outs[o] with accumulate); for the per-shift solutions of verify and of requested x_i
constexpr int kLiftOut = 8;
constexpr int kLiftMultiChunk = 64;
__global__ void __launch_bounds__(256) bs_lift_multi_kernel(const BsSlot *slots, const z64 *coef, int K, int Sst,
                                                            double2 *const *outs, int nout, int accumulate)
{
    __shared__ BsSlot sl[kLiftMultiChunk];
    __shared__ z64 cf[kLiftMultiChunk * kLiftOut];
    __shared__ double2 *op[kLiftOut];
    for (int j = threadIdx.x; j < K; j += blockDim.x) sl[j] = slots[j];
    for (int j = threadIdx.x; j < K * kLiftOut; j += blockDim.x) cf[j] = coef[j];
    if (threadIdx.x < kLiftOut) op[threadIdx.x] = (int)threadIdx.x < nout ? outs[threadIdx.x] : nullptr;
    __syncthreads();
    const int64_t np = (int64_t)6 * Sst;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < np; f += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(f / Sst), st = (int)(f - (int64_t)c2 * Sst);
        const int64_t e0 = (int64_t)(2 * c2) * Sst + st, e1 = e0 + Sst;
        z64 a0[kLiftOut], a1[kLiftOut];
#pragma unroll
        for (int o = 0; o < kLiftOut; ++o) {
            if (accumulate && o < nout) {
                a0[o] = ldz(op[o], e0);
                a1[o] = ldz(op[o], e1);
            } else {
                a0[o] = a1[o] = z64{0.0, 0.0};
            }
        }
        for (int j = 0; j < K; ++j) {
            z64 v0, v1;
            if (sl[j].f32) {
                const float4 t = static_cast<const float4 *>(sl[j].p)[f];
                v0 = {(double)t.x, (double)t.y};
                v1 = {(double)t.z, (double)t.w};
            } else {
                const double2 *q = static_cast<const double2 *>(sl[j].p);
                v0 = ldz(q, e0);
                v1 = ldz(q, e1);
            }
#pragma unroll
            for (int o = 0; o < kLiftOut; ++o) {
                const z64 c = cf[j * kLiftOut + o];
                a0[o] = a0[o] + c * v0;
                a1[o] = a1[o] + c * v1;
            }
        }
#pragma unroll
        for (int o = 0; o < kLiftOut; ++o)
            if (o < nout) {
                stz(op[o], e0, a0[o]);
                stz(op[o], e1, a1[o]);
            }
    }
}

// q = -c^2 A A x + sigma x  (for the reliable update r = y + q)
__global__ void __launch_bounds__(256) bs_addto64(const double2 *y, double2 *q, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        stz(q, e, ldz(y, e) + ldz(q, e));
}

// Lockstep batches: one descriptor per problem (device memory), the vectors in the precision of
// the problem's current phase; blockIdx.y (vector kernels) or blockIdx.x (the one-block scalar
// kernels) selects the problem.
struct BsDesc {
    BsState *S;
    void *const *rtab;
    void *const *stab;
    void *p, *v, *sv, *t, *rh;
    double2 *x64;
    z64 *spart, *vpart;
    BsHist *hist;
    int64_t n;   // complex entries (12 S)
    int Sst;
    int nb_s;    // blocks (partials) of the stencil that forms v, and of the one that forms t
    int nb_v;
    int cap;     // history capacity (maxiter)
};

__global__ void __launch_bounds__(256) bs_alpha_batch(const BsDesc *d)
{
    const BsDesc &D = d[blockIdx.x];
    bs_alpha_kernel_body(D.S, D.spart, D.nb_s);
}
__global__ void __launch_bounds__(256) bs_omega_batch(const BsDesc *d)
{
    const BsDesc &D = d[blockIdx.x];
    bs_omega_kernel_body(D.S, D.vpart, D.nb_v);
}
// nb: the grid width of the residual kernel that wrote the partials
__global__ void __launch_bounds__(256) bs_beta_batch(const BsDesc *d, int nb)
{
    const BsDesc &D = d[blockIdx.x];
    bs_beta_kernel_body(D.S, D.vpart, nb, D.hist, D.cap);
}
template <typename R>
__global__ void __launch_bounds__(256) bs_sub_batch(const BsDesc *d)
{
    using T = typename BsVec<R>::t;
    const BsDesc &D = d[blockIdx.y];
    bs_sub_stored_body<R>(D.S, D.rtab, (const T *)D.v, (T *)D.sv, D.stab, D.n);
}
template <typename R>
__global__ void __launch_bounds__(256) bs_res_batch(const BsDesc *d)
{
    using T = typename BsVec<R>::t;
    const BsDesc &D = d[blockIdx.y];
    bs_res_stored_body<R>(D.S, (const T *)D.sv, (const T *)D.t, (const T *)D.rh, D.rtab, D.n, D.vpart);
}
__global__ void __launch_bounds__(256) bs_xp64_batch(const BsDesc *d)
{
    const BsDesc &D = d[blockIdx.y];
    bs_xp64_body(D.S, (double2 *)D.p, (const double2 *)D.v, D.rtab, (const double2 *)D.sv, D.x64, D.n);
}
__global__ void __launch_bounds__(256) bs_xp32_batch(const BsDesc *d)
{
    const BsDesc &D = d[blockIdx.y];
    bs_xp32_body(D.S, (float4 *)D.p, (const float4 *)D.v, D.rtab, (const float4 *)D.sv, D.x64, D.Sst);
}

// the heads of a batch's problems into one array (one copy to the host per chunk), and back for the
// problems flagged in mask
static_assert(sizeof(BsHead) % 8 == 0, "BsHead is copied in 8-byte words");
__global__ void __launch_bounds__(64) bs_gather_heads(BsState *const *S, BsHead *out)
{
    const uint64_t *src = reinterpret_cast<const uint64_t *>(&S[blockIdx.x]->h);
    uint64_t *dst = reinterpret_cast<uint64_t *>(out + blockIdx.x);
    for (int i = threadIdx.x; i < (int)(sizeof(BsHead) / 8); i += blockDim.x) dst[i] = src[i];
}
__global__ void __launch_bounds__(64) bs_scatter_heads(BsState *const *S, const BsHead *in, const int *mask)
{
    if (!mask[blockIdx.x]) return;
    const uint64_t *src = reinterpret_cast<const uint64_t *>(in + blockIdx.x);
    uint64_t *dst = reinterpret_cast<uint64_t *>(&S[blockIdx.x]->h);
    for (int i = threadIdx.x; i < (int)(sizeof(BsHead) / 8); i += blockDim.x) dst[i] = src[i];
}

// Stored-basis slots handed out from the context's per-size pools; shared by the problems of a
// lockstep batch (each takes the next unused buffers) together with one byte budget.
struct BsSlotPools {
    std::map<size_t, size_t> next;  // next unused buffer of each per-size pool
    double budget = 0.0, used = 0.0;
};

class BsStored {
    friend class BsBatch;

  public:
    BsStored(const sgn_problem &pb, const sgn_rational &rf, const sgn_ms_opts &o, hipStream_t s,
             BsSlotPools *pools = nullptr)
        : pb_(pb), rf_(rf), o_(o), s_(s), lat_(*as_lattice(pb.lat)), ctx_(*lat_.ctx),
          pools_(pools ? pools : &own_pools_)
    {
    }
    ~BsStored()
    {
        if (gexec_) (void)hipGraphExecDestroy(gexec_);
    }
    sgn_status run(sgn_stats *stp);

  private:
    // the steps of run(): sizes, workspace bytes, setup in a given workspace (false: y = 0, the
    // result x_P is already written), the host's reaction to the device flags after a chunk of
    // iterations (true: stop), and the combination of the result
    void init_sizes();
    size_t ws_bytes() const;
    bool setup(char *ws, sgn_stats *stp);
    bool poll(BsHead &h);
    sgn_status finish(sgn_stats *stp);
    void note_launched(int count);
    const sgn_problem &pb_;
    const sgn_rational &rf_;
    const sgn_ms_opts &o_;
    hipStream_t s_;
    Lattice &lat_;
    Context &ctx_;
    int64_t n_ = 0, nc_ = 0, Sst_ = 0;
    size_t b64_ = 0, b32_ = 0;
    int ns_ = 0, seed_ = 0, nvb_ = 0, nst_ = 0, maxiter_ = 0, poll_ = 4;
    double c2_ = 0.0, s0_ = 0.0;
    // vectors (internal layouts)
    // the residual r_k lives only in its slot; r32_ is a conversion buffer
    char *y_ = nullptr, *rh64_ = nullptr, *s64_ = nullptr, *v64_ = nullptr, *t64_ = nullptr, *tmp64_ = nullptr,
         *p64_ = nullptr, *x64_ = nullptr;
    char *rh32_ = nullptr, *r32_ = nullptr, *s32_ = nullptr, *v32_ = nullptr, *t32_ = nullptr, *tmp32_ = nullptr,
         *p32_ = nullptr;
    char *rcan_ = nullptr;
    z64 *spart_ = nullptr, *vpart_ = nullptr;
    BsState *S_ = nullptr;
    BsHist *hist_ = nullptr;
    void **rtab_ = nullptr, **stab_ = nullptr;  // device slot tables (r_k, s_k)
    std::vector<void *> rslots_, sslots_;
    std::vector<char> rf32_, sf32_;
    BsSlotPools own_pools_;
    BsSlotPools *pools_;
    int phase_ = 0, launched_ = 0, reliable_ = 0;
    hipGraphExec_t gexec_ = nullptr;
    // state of run() between its steps
    std::chrono::steady_clock::time_point t_start_, t_kry_;
    double ynorm_ = 0.0;
    std::vector<double> tau_;
    sgn_status result_ = SGN_OK;
    BsHead head_{};
    bool done_ = false;

    bool lo() const { return phase_ >= 1; }
    sgn_prec sprec() const { return phase_ == 0 ? SGN_PREC_F64 : (phase_ == 1 ? SGN_PREC_F32 : SGN_PREC_F32_H16); }
    void *take_slot(size_t bytes);
    void ensure_slots(int upto);
    void launch_iteration(hipStream_t strm);
    void iterate(int count);
    void reliable_update(BsHead &h);
    // the same in two parts for a batch: the device work, with rho and ||r||^2 into out[0], out[1]
    // (device memory), then the host's update of the head from them
    void reliable_update_async(int k, z64 *out);
    void reliable_update_finish(BsHead &h, z64 rho, double nrm2);
    void switch_phase(BsHead &h, int to);
    void lift(int K, const std::vector<zc> &cr, const std::vector<zc> &cs, char *out);
    // outs[o] = the lift of (cr[o], cs[o]) for up to kLiftOut sets, one pass over the slots
    void lift_multi(int K, const std::vector<const std::vector<zc> *> &cr, const std::vector<const std::vector<zc> *> &cs,
                    const std::vector<char *> &outs);
};

// a slot buffer of the given size (FP64 or FP32 vector) from the context's pools
void *BsStored::take_slot(size_t bytes)
{
    if (pools_->used + (double)bytes > pools_->budget)
        throw Failure{SGN_ERR_NOMEM, "multishift_bicgstab: stored basis exceeds its budget (basis_slots)"};
    auto &pool = ctx_.basis_pools[bytes];
    size_t &next = pools_->next[bytes];
    if (next == pool.size()) {
        void *b = nullptr;
        if (hipMalloc(&b, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Failure{SGN_ERR_NOMEM, "multishift_bicgstab: stored basis does not fit"};
        }
        pool.push_back(b);
    }
    pools_->used += (double)bytes;
    return pool[next++];
}

// r-slots 0 .. upto + 1 and s-slots 0 .. upto; slots first written in the FP32 phase are FP32-sized
void BsStored::ensure_slots(int upto)
{
    const size_t r0 = rslots_.size(), s0 = sslots_.size();
    const size_t bytes = lo() ? b32_ : b64_;
    while ((int)rslots_.size() < upto + 2) rslots_.push_back(take_slot(bytes));
    while ((int)sslots_.size() < upto + 1) sslots_.push_back(take_slot(bytes));
    if (rslots_.size() > r0)
        SGN_HIP(hipMemcpy(rtab_ + r0, rslots_.data() + r0, sizeof(void *) * (rslots_.size() - r0),
                          hipMemcpyHostToDevice));
    if (sslots_.size() > s0)
        SGN_HIP(hipMemcpy(stab_ + s0, sslots_.data() + s0, sizeof(void *) * (sslots_.size() - s0),
                          hipMemcpyHostToDevice));
}

void BsStored::launch_iteration(hipStream_t strm)
{
    const sgn_prec sp = sprec();
    const bool f = lo();
    char *p = f ? p32_ : p64_, *tmp = f ? tmp32_ : tmp64_, *v = f ? v32_ : v64_, *sv = f ? s32_ : s64_,
         *t = f ? t32_ : t64_, *rh = f ? rh32_ : rh64_;
    OpSpec op;
    op.mu = pb_.mu;
    dslash_launch(lat_, sp, op, p, tmp, Epilogue{}, strm);
    Epilogue e2;
    e2.a = c2_;
    e2.z = p;
    e2.b = {-s0_, 0.0};
    e2.w = rh;
    e2.partials = spart_;
    const int nb = dslash_launch(lat_, sp, op, tmp, v, e2, strm);
    hipLaunchKernelGGL(bs_alpha_kernel, dim3(1), dim3(256), 0, strm, S_, (const z64 *)spart_, nb);
    const int pr = ctx_.prof_start(strm, SGN_K_SEED_UPDATE, true);
    if (f)
        launch_k(ctx_.prof_stamp(pr), bs_sub_stored<float>, dim3(nvb_), dim3(256), 0u, strm, (const BsState *)S_,
                           (void *const *)rtab_, (const float2 *)v, (float2 *)sv, (void *const *)stab_, n_);
    else
        launch_k(ctx_.prof_stamp(pr), bs_sub_stored<double>, dim3(nvb_), dim3(256), 0u, strm, (const BsState *)S_,
                           (void *const *)rtab_, (const double2 *)v, (double2 *)sv, (void *const *)stab_, n_);
    ctx_.prof_stop(pr, strm, SGN_K_SEED_UPDATE, 4.0 * (f ? 8.0 : 16.0) * n_, 8.0 * n_);
    dslash_launch(lat_, sp, op, sv, tmp, Epilogue{}, strm);
    Epilogue e4;  // t = M s with the partials of s^H t and ||t||^2
    e4.a = c2_;
    e4.z = sv;
    e4.b = {-s0_, 0.0};
    e4.w = sv;
    e4.partials = vpart_;
    e4.norm = true;
    const int nb4 = dslash_launch(lat_, sp, op, tmp, t, e4, strm);
    const double eb = f ? 8.0 : 16.0;
    int pr2 = -1;
    hipLaunchKernelGGL(bs_omega_kernel, dim3(1), dim3(256), 0, strm, S_, (const z64 *)vpart_, nb4);
    pr2 = ctx_.prof_start(strm, SGN_K_SEED_UPDATE, true);
    if (f)
        launch_k(ctx_.prof_stamp(pr2), bs_res_stored<float>, dim3(nvb_), dim3(256), 0u, strm, (const BsState *)S_,
                           (const float2 *)sv, (const float2 *)t, (const float2 *)rh, (void *const *)rtab_, n_,
                           vpart_);
    else
        launch_k(ctx_.prof_stamp(pr2), bs_res_stored<double>, dim3(nvb_), dim3(256), 0u, strm, (const BsState *)S_,
                           (const double2 *)sv, (const double2 *)t, (const double2 *)rh, (void *const *)rtab_, n_,
                           vpart_);
    ctx_.prof_stop(pr2, strm, SGN_K_SEED_UPDATE, 4.0 * eb * n_, 12.0 * n_);
    hipLaunchKernelGGL(bs_beta_kernel, dim3(1), dim3(256), 0, strm, S_, (const z64 *)vpart_, nvb_, hist_, maxiter_);
    const int pr3 = ctx_.prof_start(strm, SGN_K_SHIFT_UPDATE, true);
    if (f)
        launch_k(ctx_.prof_stamp(pr3), bs_xp32, dim3(vec_blocks(6 * Sst_)), dim3(256), 0u, strm, (const BsState *)S_, (float4 *)p,
                           (const float4 *)v, (void *const *)rtab_, (const float4 *)sv, (double2 *)x64_, (int)Sst_);
    else
        launch_k(ctx_.prof_stamp(pr3), bs_xp64, dim3(nvb_), dim3(256), 0u, strm, (const BsState *)S_, (double2 *)p,
                           (const double2 *)v, (void *const *)rtab_, (const double2 *)sv, (double2 *)x64_, n_);
    ctx_.prof_stop(pr3, strm, SGN_K_SHIFT_UPDATE, (5.0 * eb + 32.0) * n_, 28.0 * n_);
    SGN_HIP(hipGetLastError());
}

void BsStored::iterate(int count)
{
    replay_or_capture(ctx_, gexec_, o_.graph >= 0, s_, [&](hipStream_t strm) {
        for (int it = 0; it < count; ++it) launch_iteration(strm);
    });
    note_launched(count);
}

void BsStored::note_launched(int count)
{
    for (int it = 0; it < count; ++it) {  // slot precision of the iterations just launched
        const int k = launched_ + it;
        if ((int)sf32_.size() <= k) sf32_.resize(k + 1, 0);
        if ((int)rf32_.size() <= k + 1) rf32_.resize(k + 2, 0);
        sf32_[k] = lo() ? 1 : 0;
        rf32_[k + 1] = lo() ? 1 : 0;
    }
    launched_ += count;
}

// r = y - (c^2 A^2 - sigma_seed) x in FP64; it replaces the
// residual of the current iteration in its slot (in the FP32 phase); rho, the residual norm
// and its running maximum restart from it
void BsStored::reliable_update(BsHead &h)
{
    OpSpec op;
    op.mu = pb_.mu;
    dslash_launch(lat_, SGN_PREC_F64, op, x64_, tmp64_, Epilogue{}, s_);
    Epilogue ep;
    ep.a = -c2_;
    ep.z = x64_;
    ep.b = {s0_, 0.0};
    dslash_launch(lat_, SGN_PREC_F64, op, tmp64_, t64_, ep, s_);
    hipLaunchKernelGGL(bs_addto64, dim3(nvb_), dim3(256), 0, s_, (const double2 *)y_, (double2 *)t64_, n_);
    SGN_HIP(hipGetLastError());
    const int k = h.iter;
    convert_64_to_32(t64_, r32_, Sst_, s_);
    SGN_HIP(hipMemcpyAsync(rslots_[k], r32_, b32_, hipMemcpyDeviceToDevice, s_));
    rf32_[k] = 1;
    h.rho = dot_sync(ctx_, rh32_, r32_, n_, true, s_);
    h.rnorm = norm_sync(ctx_, r32_, n_, true, s_);
    h.rmax = h.rnorm;
    h.reliable = 0;
    ++reliable_;
}

void BsStored::reliable_update_async(int k, z64 *out)
{
    OpSpec op;
    op.mu = pb_.mu;
    dslash_launch(lat_, SGN_PREC_F64, op, x64_, tmp64_, Epilogue{}, s_);
    Epilogue ep;
    ep.a = -c2_;
    ep.z = x64_;
    ep.b = {s0_, 0.0};
    dslash_launch(lat_, SGN_PREC_F64, op, tmp64_, t64_, ep, s_);
    hipLaunchKernelGGL(bs_addto64, dim3(nvb_), dim3(256), 0, s_, (const double2 *)y_, (double2 *)t64_, n_);
    SGN_HIP(hipGetLastError());
    convert_64_to_32(t64_, r32_, Sst_, s_);
    SGN_HIP(hipMemcpyAsync(rslots_[k], r32_, b32_, hipMemcpyDeviceToDevice, s_));
    rf32_[k] = 1;
    // the same reductions as dot_sync / norm_sync, left on the device (stream order lets the
    // context's partials be reused by the next problem)
    z64 *part = static_cast<z64 *>(ctx_.ensure_partials((kMaxBlocks + 1) * sizeof(z64)));
    int nb = dot_partials(rh32_, r32_, n_, true, part, s_);
    finalize_sum(part, nb, out, s_);
    nb = norm2_partials(r32_, n_, true, part, s_);
    finalize_sum(part, nb, out + 1, s_);
}

void BsStored::reliable_update_finish(BsHead &h, z64 rho, double nrm2)
{
    h.rho = rho;
    h.rnorm = std::sqrt(nrm2);
    h.rmax = h.rnorm;
    h.reliable = 0;
    ++reliable_;
    head_ = h;
}

void BsStored::switch_phase(BsHead &h, int to)
{
    if (phase_ == 0 && to >= 1) {
        // the current residual's slot becomes FP32 (what the FP32 iteration reads); p and the
        // shadow vector move to FP32
        const int k = h.iter;
        convert_64_to_32(rslots_[k], r32_, Sst_, s_);
        SGN_HIP(hipMemcpyAsync(rslots_[k], r32_, b32_, hipMemcpyDeviceToDevice, s_));
        rf32_[k] = 1;
        convert_64_to_32(p64_, p32_, Sst_, s_);
        convert_64_to_32(rh64_, rh32_, Sst_, s_);
        h.rho = dot_sync(ctx_, rh32_, r32_, n_, true, s_);
        h.rnorm = norm_sync(ctx_, r32_, n_, true, s_);
        h.rmax = h.rnorm;
    }
    phase_ = to;
    h.phase = to;
    h.want_phase = 0;
    if (gexec_) {
        (void)hipGraphExecDestroy(gexec_);
        gexec_ = nullptr;
    }
}

// out += sum_j cr_j r_j + sum_j cs_j s_j over the stored slots (r_0..r_K, s_0..s_{K-1})
void BsStored::lift(int K, const std::vector<zc> &cr, const std::vector<zc> &cs, char *out)
{
    std::vector<BsSlot> sl;
    std::vector<z64> cf;
    for (int j = 0; j <= K; ++j) {
        sl.push_back(BsSlot{rslots_[j], j < (int)rf32_.size() ? rf32_[j] : 0, 0});
        cf.push_back({cr[j].real(), cr[j].imag()});
    }
    for (int j = 0; j < K; ++j) {
        sl.push_back(BsSlot{sslots_[j], j < (int)sf32_.size() ? sf32_[j] : 0, 0});
        cf.push_back({cs[j].real(), cs[j].imag()});
    }
    const int nk = (int)sl.size();
    DeviceScratch dsl(sizeof(BsSlot) * nk), dcf(sizeof(z64) * nk);
    SGN_HIP(hipMemcpy(dsl.p, sl.data(), sizeof(BsSlot) * nk, hipMemcpyHostToDevice));
    SGN_HIP(hipMemcpy(dcf.p, cf.data(), sizeof(z64) * nk, hipMemcpyHostToDevice));
    const int pr = ctx_.prof_start(s_, SGN_K_LIFT);
    double bytes = 2.0 * b64_;
    for (int j = 0; j < nk; ++j) bytes += sl[j].f32 ? (double)b32_ : (double)b64_;
    for (int j0 = 0; j0 < nk; j0 += kBsLiftChunk)
        hipLaunchKernelGGL(bs_lift_kernel, dim3(vec_blocks(6 * Sst_)), dim3(256), 0, s_,
                           static_cast<const BsSlot *>(dsl.p) + j0, static_cast<const z64 *>(dcf.p) + j0,
                           std::min(kBsLiftChunk, nk - j0), (int)Sst_, (double2 *)out);
    ctx_.prof_stop(pr, s_, SGN_K_LIFT, bytes, 8.0 * nk * (double)n_);
    SGN_HIP(hipGetLastError());
    SGN_HIP(hipStreamSynchronize(s_));  // before the coefficient buffers are freed
}

void BsStored::lift_multi(int K, const std::vector<const std::vector<zc> *> &cr,
                          const std::vector<const std::vector<zc> *> &cs, const std::vector<char *> &outs)
{
    const int nout = (int)outs.size();
    SGN_REQUIRE(nout >= 1 && nout <= kLiftOut && (int)cr.size() == nout && (int)cs.size() == nout,
                "multishift_bicgstab: lift sets");
    std::vector<BsSlot> sl;
    for (int j = 0; j <= K; ++j) sl.push_back(BsSlot{rslots_[j], j < (int)rf32_.size() ? rf32_[j] : 0, 0});
    for (int j = 0; j < K; ++j) sl.push_back(BsSlot{sslots_[j], j < (int)sf32_.size() ? sf32_[j] : 0, 0});
    const int nk = (int)sl.size();
    std::vector<z64> cf((size_t)nk * kLiftOut, z64{0.0, 0.0});
    for (int o = 0; o < nout; ++o) {
        for (int j = 0; j <= K; ++j) cf[(size_t)j * kLiftOut + o] = {(*cr[o])[j].real(), (*cr[o])[j].imag()};
        for (int j = 0; j < K; ++j)
            cf[(size_t)(K + 1 + j) * kLiftOut + o] = {(*cs[o])[j].real(), (*cs[o])[j].imag()};
    }
    DeviceScratch dsl(sizeof(BsSlot) * nk), dcf(sizeof(z64) * cf.size()), dout(sizeof(void *) * kLiftOut);
    SGN_HIP(hipMemcpy(dsl.p, sl.data(), sizeof(BsSlot) * nk, hipMemcpyHostToDevice));
    SGN_HIP(hipMemcpy(dcf.p, cf.data(), sizeof(z64) * cf.size(), hipMemcpyHostToDevice));
    SGN_HIP(hipMemcpy(dout.p, outs.data(), sizeof(void *) * nout, hipMemcpyHostToDevice));
    const int pr = ctx_.prof_start(s_, SGN_K_LIFT);
    double bytes = 2.0 * nout * b64_;
    for (int j = 0; j < nk; ++j) bytes += sl[j].f32 ? (double)b32_ : (double)b64_;
    for (int j0 = 0; j0 < nk; j0 += kLiftMultiChunk)
        hipLaunchKernelGGL(bs_lift_multi_kernel, dim3(vec_blocks(6 * Sst_)), dim3(256), 0, s_,
                           static_cast<const BsSlot *>(dsl.p) + j0,
                           static_cast<const z64 *>(dcf.p) + (size_t)j0 * kLiftOut, std::min(kLiftMultiChunk, nk - j0),
                           (int)Sst_, static_cast<double2 *const *>(dout.p), nout, j0 > 0 ? 1 : 0);
    ctx_.prof_stop(pr, s_, SGN_K_LIFT, bytes, 8.0 * nk * nout * (double)n_);
    SGN_HIP(hipGetLastError());
    SGN_HIP(hipStreamSynchronize(s_));  // before the coefficient buffers are freed
}

void BsStored::init_sizes()
{
    ns_ = rf_.s;
    Sst_ = lat_.S;
    n_ = 12 * lat_.S;
    nc_ = 12 * lat_.V;
    b64_ = (size_t)n_ * 16;
    b32_ = (size_t)n_ * 8;
    nvb_ = vec_blocks(n_);
    nst_ = dslash_blocks(lat_);
    maxiter_ = o_.maxiter > 0 ? o_.maxiter : 10000;
    poll_ = o_.poll > 0 ? o_.poll : 4;
    for (int i = 1; i < ns_; ++i)
        if (std::abs(rf_.sigma[i]) < std::abs(rf_.sigma[seed_])) seed_ = i;
    s0_ = rf_.sigma[seed_];
    c2_ = rf_.c * rf_.c;
}

// partials: the dotting stencils' (nst_ blocks, two per block for the second one) and the vector kernels'
size_t BsStored::ws_bytes() const
{
    const bool mixed = o_.prec != SGN_PREC_F64;
    const size_t nvp = 2 * (size_t)std::max(nst_, kMaxBlocks);
    const size_t scal = sizeof(z64) * ((size_t)nst_ + nvp) + sizeof(BsState) + sizeof(BsHist) * (size_t)maxiter_ +
                        2 * sizeof(void *) * ((size_t)maxiter_ + poll_ + 4);
    return (8 * b64_ + (mixed ? 7 * b32_ : 0) + (size_t)nc_ * 16 + scal + 512 + 255) / 256 * 256;
}

bool BsStored::setup(char *a, sgn_stats *stp)
{
    t_start_ = std::chrono::steady_clock::now();
    SGN_HIP(hipSetDevice(ctx_.device));
    const bool mixed = o_.prec != SGN_PREC_F64;
    const size_t c64 = (size_t)nc_ * 16;
    const size_t nvp = 2 * (size_t)std::max(nst_, kMaxBlocks);
    char *q = a;
    for (char **v : {&y_, &rh64_, &s64_, &v64_, &t64_, &tmp64_, &p64_, &x64_}) {
        *v = q;
        q += b64_;
    }
    if (mixed)
        for (char **v : {&rh32_, &r32_, &s32_, &v32_, &t32_, &tmp32_, &p32_}) {
            *v = q;
            q += b32_;
        }
    rcan_ = q;
    q += c64;
    q = reinterpret_cast<char *>(((uintptr_t)q + 255) & ~(uintptr_t)255);
    spart_ = reinterpret_cast<z64 *>(q);
    vpart_ = spart_ + nst_;
    S_ = reinterpret_cast<BsState *>(vpart_ + nvp);
    hist_ = reinterpret_cast<BsHist *>(S_ + 1);
    rtab_ = reinterpret_cast<void **>(hist_ + maxiter_);
    stab_ = rtab_ + maxiter_ + poll_ + 2;
    // stored-basis budget: basis_slots > 0 FP64-sized vectors, else up to half of the free device
    // memory (counting the pooled buffers as free); a batch sets it once for all its problems
    if (pools_ == &own_pools_) {
        size_t fr = 0, tot = 0;
        SGN_HIP(hipMemGetInfo(&fr, &tot));
        double held = 0.0;
        for (auto &kv : ctx_.basis_pools) held += (double)kv.first * kv.second.size();
        pools_->budget = o_.basis_slots > 0 ? (double)o_.basis_slots * b64_ : 0.5 * ((double)fr + held);
    }
    OpSpec op;
    op.mu = pb_.mu;
    // x = x_P, y = c H (I - P) b
    deflation_prologue(ctx_, pb_.defl, nc_, pb_.b, pb_.x, rcan_, nullptr, s_);
    pack_spinor(lat_, rcan_, tmp64_, SGN_PREC_F64, s_);
    {
        Epilogue ep;
        ep.a = rf_.c;
        dslash_launch(lat_, SGN_PREC_F64, op, tmp64_, y_, ep, s_);
    }
    ynorm_ = norm_sync(ctx_, y_, n_, false, s_);
    SGN_REQUIRE(std::isfinite(ynorm_), "multishift_bicgstab: b contains NaN or Inf");
    if (ynorm_ == 0.0) {
        SGN_HIP(hipStreamSynchronize(s_));
        if (stp) {
            *stp = sgn_stats{};
            stp->nshift = ns_;
        }
        done_ = true;
        return false;
    }
    ensure_slots(poll_);
    rf32_.assign(1, 0);
    for (char *v : {rh64_, p64_}) SGN_HIP(hipMemcpyAsync(v, y_, b64_, hipMemcpyDeviceToDevice, s_));
    SGN_HIP(hipMemcpyAsync(rslots_[0], y_, b64_, hipMemcpyDeviceToDevice, s_));
    hipLaunchKernelGGL(bs_fill_kernel<double2>, dim3(nvb_), dim3(256), 0, s_, (double2 *)x64_, make_double2(0.0, 0.0),
                       n_);
    SGN_HIP(hipGetLastError());
    tau_.assign(ns_, 0.0);
    BsState h0{};
    h0.h.rho = {ynorm_ * ynorm_, 0.0};
    h0.h.alpha_prev = {1.0, 0.0};
    h0.h.rnorm = h0.h.rmax = h0.h.ynorm = ynorm_;
    h0.h.tol = o_.tol;
    h0.h.delta = o_.delta > 0 ? o_.delta : 0.1;
    h0.h.theta32 = mixed ? (o_.theta32 > 0 ? o_.theta32 : 1e-3) : 0.0;
    const bool deflated = pb_.defl && pb_.defl->m > 0;  // FP16 links would excite the deflated modes
    h0.h.theta16 = (o_.prec == SGN_PREC_F32_H16 && !deflated) ? (o_.theta16 > 0 ? o_.theta16 : 1e-6) : 0.0;
    h0.h.maxiter = maxiter_;
    h0.h.ns = ns_;
    h0.h.seed = seed_;
    for (int i = 0; i < ns_; ++i) {
        tau_[i] = s0_ - rf_.sigma[i];
        h0.zeta[i] = h0.zeta_prev[i] = h0.zeta_next[i] = h0.pi[i] = {1.0, 0.0};
        h0.tau[i] = tau_[i];
        h0.act[i] = 1;
    }
    SGN_HIP(hipMemcpyAsync(S_, &h0, sizeof(BsState), hipMemcpyHostToDevice, s_));
    SGN_HIP(hipStreamSynchronize(s_));
    t_kry_ = std::chrono::steady_clock::now();
    return true;
}

// h: the device head just read after a chunk of iterations; a reliable update or a precision
// switch it asks for is done here (and the head written back)
bool BsStored::poll(BsHead &h)
{
    head_ = h;
    if (h.breakdown) {
        result_ = SGN_ERR_BREAKDOWN;
        done_ = true;
        return true;
    }
    if (h.done) {
        if (h.iter >= maxiter_) {
            // converged in the last iteration or not at all: decided from the estimates in finish()
            result_ = SGN_ERR_NOT_CONVERGED;
        }
        done_ = true;
        return true;
    }
    bool changed = false;
    if (h.reliable) {
        reliable_update(h);
        changed = true;
    }
    if (h.want_phase) {
        switch_phase(h, h.want_phase);
        changed = true;
    }
    if (changed) {
        SGN_HIP(hipMemcpyAsync(&S_->h, &h, sizeof(BsHead), hipMemcpyHostToDevice, s_));
        SGN_HIP(hipStreamSynchronize(s_));
    }
    head_ = h;
    return false;
}

sgn_status BsStored::run(sgn_stats *stp)
{
    init_sizes();
    if (!setup(static_cast<char *>(ctx_.ensure_arena(ws_bytes())), stp)) return SGN_OK;
    for (;;) {
        ensure_slots(launched_ + poll_);
        iterate(poll_);
        BsHead h{};
        SGN_HIP(hipMemcpyAsync(&h, &S_->h, sizeof(BsHead), hipMemcpyDeviceToHost, s_));
        SGN_HIP(hipStreamSynchronize(s_));
        if (poll(h)) break;
    }
    return finish(stp);
}

sgn_status BsStored::finish(sgn_stats *stp)
{
    const BsHead &h = head_;
    const double ynorm = ynorm_;
    const std::vector<double> &tau = tau_;
    sgn_status result = result_;
    sgn_stats st{};
    st.nshift = ns_;
    OpSpec op;
    op.mu = pb_.mu;
    const int K = h.iter;
    // coefficients of sum_{i != seed} omega_i x_i over the slots r_0..r_K, s_0..s_{K-1}
    std::vector<BsHist> hs(K);
    if (K) SGN_HIP(hipMemcpy(hs.data(), hist_, sizeof(BsHist) * K, hipMemcpyDeviceToHost));
    const double lim = o_.tol * ynorm;
    std::vector<zc> dr(K + 1, 0.0), ds(K, 0.0);
    std::vector<std::vector<zc>> xr_i, xs_i;  // per-shift coefficients when the x_i are requested or verified
    if (pb_.x_shift || o_.verify) {
        xr_i.resize(ns_);
        xs_i.resize(ns_);
    }
    double worst = 0.0;
    for (int i = 0; i < ns_; ++i) {
        zc zeta = 1.0, zeta_prev = 1.0, pi = 1.0, ap = 1.0, bp = 0.0;
        std::vector<zc> Pr(K + 1, 0.0), Ps(K, 0.0), Xr(K + 1, 0.0), Xs(K, 0.0);
        Pr[0] = 1.0;
        bool frozen = false;
        double res = 1.0;
        for (int k = 0; k < K && !frozen; ++k) {
            const zc al(hs[k].alpha.r, hs[k].alpha.i), om(hs[k].omega.r, hs[k].omega.i), be(hs[k].beta.r, hs[k].beta.i);
            const zc zn = zeta * zeta_prev * ap / (ap * (1.0 + tau[i] * al) * zeta_prev + al * bp * (zeta_prev - zeta));
            const zc ai = al * zn / zeta, qq = zn / zeta, bi = be * qq * qq, oi = om / (1.0 + om * tau[i]);
            const zc pn = pi * (1.0 + om * tau[i]);
            const zc ks = (std::abs(ai) > 0.0) ? bi * oi / ai : zc(0.0, 0.0);
            for (int j = 0; j <= k; ++j) {
                Xr[j] += ai * Pr[j];
                if (j < k) Xs[j] += ai * Ps[j];
            }
            Xs[k] += oi * zn / pi;
            for (int j = 0; j <= k; ++j) {
                Pr[j] *= bi;
                if (j < k) Ps[j] *= bi;
            }
            Pr[k] += -ks * zeta / pi;
            Ps[k] = ks * zn / pi;
            Pr[k + 1] = zn / pn;
            zeta_prev = zeta;
            zeta = zn;
            pi = pn;
            ap = al;
            bp = be;
            res = std::abs(zeta / pi) * hs[k].rnorm;
            if (i != seed_ && res <= lim) frozen = true;
        }
        if (K == 0) res = ynorm;
        st.shift_residual[i] = res / ynorm;
        worst = std::max(worst, st.shift_residual[i]);
        if (i == seed_) continue;
        if (pb_.x_shift || o_.verify) {
            xr_i[i] = Xr;
            xs_i[i] = Xs;
        }
        for (int j = 0; j <= K; ++j) dr[j] += rf_.omega[i] * Xr[j];
        for (int j = 0; j < K; ++j) ds[j] += rf_.omega[i] * Xs[j];
    }
    if (result == SGN_ERR_NOT_CONVERGED && worst <= o_.tol) result = SGN_OK;
    int refine_its = 0, extra_mv = 0;
    if (o_.verify) {
        // every shifted solution explicitly (one lift each), its FP64 true residual, and an FP64
        // refinement of any system above the tolerance; x = x_P + sum_i omega_i x_i of the checked
        // x_i.  Work fields: the iteration's FP64 vectors (free after the loop) plus six more.
        char *acc = p64_, *res = v64_, *tmp = t64_;
        std::unique_ptr<DeviceScratch> work;
        hipLaunchKernelGGL(bs_fill_kernel<double2>, dim3(nvb_), dim3(256), 0, s_, (double2 *)acc,
                           make_double2(0.0, 0.0), n_);
        SGN_HIP(hipGetLastError());
        worst = 0.0;
        // the seed's x first, then the other shifts' x_i lifted kLiftOut at a time in one pass
        std::vector<int> order{seed_};
        for (int i = 0; i < ns_; ++i)
            if (i != seed_) order.push_back(i);
        DeviceScratch xbuf((size_t)kLiftOut * b64_);
        for (size_t g0 = 0; g0 < order.size(); g0 += (g0 == 0 ? 1 : kLiftOut)) {
            const size_t g1 = g0 == 0 ? 1 : std::min(order.size(), g0 + kLiftOut);
            std::vector<char *> outs;
            for (size_t q = g0; q < g1; ++q) outs.push_back(static_cast<char *>(xbuf.p) + (q - g0) * b64_);
            if (g0 == 0) {
                SGN_HIP(hipMemcpyAsync(outs[0], x64_, b64_, hipMemcpyDeviceToDevice, s_));
            } else {
                std::vector<const std::vector<zc> *> cr, cs;
                for (size_t q = g0; q < g1; ++q) {
                    cr.push_back(&xr_i[order[q]]);
                    cs.push_back(&xs_i[order[q]]);
                }
                lift_multi(K, cr, cs, outs);
            }
            for (size_t q = g0; q < g1; ++q) {
                const int i = order[q];
                char *xi = outs[q - g0];
                double ri = shift_residual64(lat_, op, c2_, rf_.sigma[i], y_, xi, res, tmp, s_) / ynorm;
                extra_mv += 2;
                if (ri > o_.tol) {
                    if (!work) work = std::make_unique<DeviceScratch>(6 * b64_);
                    refine_its += refine_shift64(lat_, op, c2_, rf_.sigma[i], res, xi, 0.5 * o_.tol * ynorm, maxiter_,
                                                 work->p, tmp, s_, &extra_mv);
                    ri = shift_residual64(lat_, op, c2_, rf_.sigma[i], y_, xi, res, tmp, s_) / ynorm;
                    extra_mv += 2;
                }
                st.shift_residual[i] = ri;
                worst = std::max(worst, ri);
                axpby64({rf_.omega[i], 0.0}, xi, {1.0, 0.0}, acc, n_, s_);
                if (pb_.x_shift && pb_.x_shift[i]) unpack_spinor(lat_, xi, pb_.x_shift[i], SGN_PREC_F64, s_);
            }
        }
        SGN_HIP(hipStreamSynchronize(s_));  // the lifted x_i are read until here
        result = worst <= o_.tol ? (result == SGN_ERR_NOT_CONVERGED ? SGN_OK : result) : SGN_ERR_NOT_CONVERGED;
        unpack_spinor(lat_, acc, rcan_, SGN_PREC_F64, s_);
    } else {
        // x_int = omega_seed x_seed + lift
        scale64({rf_.omega[seed_], 0.0}, x64_, tmp64_, n_, s_);
        lift(K, dr, ds, tmp64_);
        unpack_spinor(lat_, tmp64_, rcan_, SGN_PREC_F64, s_);
    }
    if (pb_.defl && pb_.defl->m > 0) {  // the exact x_i lie in range(I - P): drop rounding components
        DeviceScratch cd(sizeof(z64) * pb_.defl->m);
        deflate_dots(pb_.defl->L, pb_.defl->m, rcan_, nc_, static_cast<z64 *>(cd.p), ctx_, s_);
        deflate_combine(rcan_, {1.0, 0.0}, {-1.0, 0.0}, pb_.defl->R, pb_.defl->m, static_cast<const z64 *>(cd.p),
                        nullptr, nc_, s_);
        SGN_HIP(hipStreamSynchronize(s_));
    }
    axpby64({1.0, 0.0}, rcan_, {1.0, 0.0}, pb_.x, nc_, s_);
    if (pb_.x_shift && !o_.verify)  // each shift's own solution (the seed's is x itself)
        for (int i = 0; i < ns_; ++i) {
            if (!pb_.x_shift[i]) continue;
            if (i == seed_) {
                SGN_HIP(hipMemcpyAsync(tmp64_, x64_, b64_, hipMemcpyDeviceToDevice, s_));
            } else {
                hipLaunchKernelGGL(bs_fill_kernel<double2>, dim3(nvb_), dim3(256), 0, s_, (double2 *)tmp64_,
                                   make_double2(0.0, 0.0), n_);
                SGN_HIP(hipGetLastError());
                lift(K, xr_i[i], xs_i[i], tmp64_);
            }
            unpack_spinor(lat_, tmp64_, pb_.x_shift[i], SGN_PREC_F64, s_);
        }
    SGN_HIP(hipStreamSynchronize(s_));
    st.iterations = K;
    st.matvecs = 4 * K + 1 + 2 * reliable_ + extra_mv;
    st.reliable_updates = reliable_;
    st.refine_iterations = refine_its;
    st.residual = worst;
    st.krylov_ms = ms_since(t_kry_);
    st.total_ms = ms_since(t_start_);
    if (stp) *stp = st;
    return result;
}

// Lockstep batch of stored-basis problems (own lattices, mu and b; one rational function):
// every iteration of all active problems is one set of launches per precision phase -- the four
// stencil applications as StencilBatch launches (problems on one lattice share their link loads in
// multi-RHS groups), the scalar steps one block per problem, the vector updates with blockIdx.y over
// the problems -- and a chunk of poll iterations is captured once as a HIP graph and replayed until
// a problem changes precision or several have finished.  Setup, reliable updates, precision switches
// and the final combination are each problem's own (BsStored's steps).
class BsBatch {
  public:
    BsBatch(const sgn_problem *pb, int np, const sgn_rational &rf, const sgn_ms_opts &o, hipStream_t s)
        : o_(o), s_(s)
    {
        for (int k = 0; k < np; ++k) {
            SGN_REQUIRE(pb[k].lat && pb[k].b && pb[k].x, "multishift_bicgstab: null problem field");
            SGN_REQUIRE(std::isfinite(pb[k].mu), "multishift_bicgstab: mu not finite");
            pr_.push_back(std::make_unique<BsStored>(pb[k], rf, o, s, &pools_));
        }
        ctx_ = pr_.empty() ? nullptr : &pr_[0]->ctx_;
        for (auto &p : pr_) SGN_REQUIRE(&p->ctx_ == ctx_, "multishift_bicgstab: problems of one call need one context");
    }
    ~BsBatch()
    {
        drop_graph();
        for (BsDesc *d : ddesc_)
            if (d) (void)hipFree(d);
        if (hpin_) (void)hipHostFree(hpin_);
        if (hru_) (void)hipHostFree(hru_);
    }
    sgn_status run(sgn_stats *st);

  private:
    std::vector<std::unique_ptr<BsStored>> pr_;
    BsSlotPools pools_;
    const sgn_ms_opts &o_;
    hipStream_t s_;
    Context *ctx_ = nullptr;
    int poll_ = 4;
    std::vector<int> group_[3];          // active problems of each phase
    BsDesc *ddesc_[3] = {nullptr, nullptr, nullptr};
    size_t dcap_[3] = {0, 0, 0};
    StencilBatch stb_[3][4];
    int nvb_max_[3] = {0, 0, 0}, nxp_max_[3] = {0, 0, 0};
    double vbytes_[3] = {0, 0, 0};       // bytes of one element pass of every problem of the phase
    hipGraphExec_t gexec_ = nullptr;
    // host <-> device traffic of the polls: the problems' state pointers, their heads gathered in
    // device memory, a pinned host mirror (heads, then the write-back mask), the reliable updates'
    // reductions (two per problem) and their pinned mirror
    std::unique_ptr<DeviceScratch> dsptr_, dheads_, dru_;
    char *hpin_ = nullptr;
    z64 *hru_ = nullptr;

    void drop_graph()
    {
        if (gexec_) (void)hipGraphExecDestroy(gexec_);
        gexec_ = nullptr;
    }
    void rebuild();
    void launch_iteration(hipStream_t strm);
    void iterate(int count);
};

void BsBatch::rebuild()
{
    drop_graph();
    for (auto &g : group_) g.clear();
    for (int k = 0; k < (int)pr_.size(); ++k)
        if (!pr_[k]->done_) group_[pr_[k]->phase_].push_back(k);
    for (int ph = 0; ph < 3; ++ph) {
        const std::vector<int> &g = group_[ph];
        std::vector<StencilJob> jobs[4];
        std::vector<BsDesc> desc(g.size());
        nvb_max_[ph] = nxp_max_[ph] = 0;
        vbytes_[ph] = 0.0;
        for (size_t j = 0; j < g.size(); ++j) {
            BsStored &b = *pr_[g[j]];
            const bool f = b.lo();
            char *p = f ? b.p32_ : b.p64_, *tmp = f ? b.tmp32_ : b.tmp64_, *v = f ? b.v32_ : b.v64_,
                 *sv = f ? b.s32_ : b.s64_, *t = f ? b.t32_ : b.t64_, *rh = f ? b.rh32_ : b.rh64_;
            OpSpec op;
            op.mu = b.pb_.mu;
            jobs[0].push_back(StencilJob{&b.lat_, op, p, tmp, Epilogue{}});
            StencilJob j2{&b.lat_, op, tmp, v, Epilogue{}};
            j2.ep.a = b.c2_;
            j2.ep.z = p;
            j2.ep.b = {-b.s0_, 0.0};
            j2.ep.w = rh;
            j2.ep.partials = b.spart_;
            jobs[1].push_back(j2);
            jobs[2].push_back(StencilJob{&b.lat_, op, sv, tmp, Epilogue{}});
            StencilJob j4{&b.lat_, op, tmp, t, Epilogue{}};
            j4.ep.a = b.c2_;
            j4.ep.z = sv;
            j4.ep.b = {-b.s0_, 0.0};
            j4.ep.w = sv;
            j4.ep.partials = b.vpart_;
            j4.ep.norm = true;
            jobs[3].push_back(j4);
            desc[j] = BsDesc{b.S_, b.rtab_, b.stab_, p, v, sv, t, rh, (double2 *)b.x64_, b.spart_, b.vpart_,
                             b.hist_, b.n_, (int)b.Sst_, 0, 0, b.maxiter_};
            nvb_max_[ph] = std::max(nvb_max_[ph], b.nvb_);
            nxp_max_[ph] = std::max(nxp_max_[ph], f ? vec_blocks(6 * b.Sst_) : b.nvb_);
            vbytes_[ph] += (double)b.n_ * (f ? 8.0 : 16.0);
        }
        const sgn_prec sp = ph == 0 ? SGN_PREC_F64 : (ph == 1 ? SGN_PREC_F32 : SGN_PREC_F32_H16);
        for (int k = 0; k < 4; ++k) stb_[ph][k].prepare(jobs[k], sp);
        for (size_t j = 0; j < g.size(); ++j) {
            desc[j].nb_s = stb_[ph][1].blocks(j);
            desc[j].nb_v = stb_[ph][3].blocks(j);
        }
        if (g.empty()) continue;
        const size_t need = sizeof(BsDesc) * g.size();
        if (need > dcap_[ph]) {
            if (ddesc_[ph]) SGN_HIP(hipFree(ddesc_[ph]));
            ddesc_[ph] = nullptr;
            dcap_[ph] = 0;
            if (hipMalloc(&ddesc_[ph], need) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "multishift_bicgstab: batch"};
            dcap_[ph] = need;
        }
        SGN_HIP(hipMemcpy(ddesc_[ph], desc.data(), need, hipMemcpyHostToDevice));
    }
}

void BsBatch::launch_iteration(hipStream_t strm)
{
    for (int ph = 0; ph < 3; ++ph) {
        const int np = (int)group_[ph].size();
        if (!np) continue;
        const BsDesc *d = ddesc_[ph];
        const bool f = ph >= 1;
        const double nvec = vbytes_[ph] / (f ? 8.0 : 16.0);  // complex entries of all the phase's problems
        stb_[ph][0].launch(strm);
        stb_[ph][1].launch(strm);
        hipLaunchKernelGGL(bs_alpha_batch, dim3(np), dim3(256), 0, strm, d);
        int pr = ctx_->prof_start(strm, SGN_K_SEED_UPDATE, true);
        if (f)
            launch_k(ctx_->prof_stamp(pr), bs_sub_batch<float>, dim3(nvb_max_[ph], np), dim3(256), 0u, strm, d);
        else
            launch_k(ctx_->prof_stamp(pr), bs_sub_batch<double>, dim3(nvb_max_[ph], np), dim3(256), 0u, strm, d);
        ctx_->prof_stop(pr, strm, SGN_K_SEED_UPDATE, 4.0 * vbytes_[ph], 8.0 * nvec);
        stb_[ph][2].launch(strm);
        stb_[ph][3].launch(strm);
        hipLaunchKernelGGL(bs_omega_batch, dim3(np), dim3(256), 0, strm, d);
        pr = ctx_->prof_start(strm, SGN_K_SEED_UPDATE, true);
        if (f)
            launch_k(ctx_->prof_stamp(pr), bs_res_batch<float>, dim3(nvb_max_[ph], np), dim3(256), 0u, strm, d);
        else
            launch_k(ctx_->prof_stamp(pr), bs_res_batch<double>, dim3(nvb_max_[ph], np), dim3(256), 0u, strm, d);
        ctx_->prof_stop(pr, strm, SGN_K_SEED_UPDATE, 4.0 * vbytes_[ph], 12.0 * nvec);
        hipLaunchKernelGGL(bs_beta_batch, dim3(np), dim3(256), 0, strm, d, nvb_max_[ph]);
        pr = ctx_->prof_start(strm, SGN_K_SHIFT_UPDATE, true);
        if (f)
            launch_k(ctx_->prof_stamp(pr), bs_xp32_batch, dim3(nxp_max_[ph], np), dim3(256), 0u, strm, d);
        else
            launch_k(ctx_->prof_stamp(pr), bs_xp64_batch, dim3(nvb_max_[ph], np), dim3(256), 0u, strm, d);
        ctx_->prof_stop(pr, strm, SGN_K_SHIFT_UPDATE, 5.0 * vbytes_[ph] + 32.0 * nvec, 28.0 * nvec);
    }
    SGN_HIP(hipGetLastError());
}

void BsBatch::iterate(int count)
{
    replay_or_capture(*ctx_, gexec_, o_.graph >= 0, s_, [&](hipStream_t strm) {
        for (int it = 0; it < count; ++it) launch_iteration(strm);
    });
    for (int ph = 0; ph < 3; ++ph)
        for (int k : group_[ph]) pr_[k]->note_launched(count);
}

sgn_status BsBatch::run(sgn_stats *st)
{
    if (pr_.empty()) return SGN_OK;
    SGN_HIP(hipSetDevice(ctx_->device));
    size_t total = 0;
    double b64sum = 0.0;
    for (auto &p : pr_) {
        p->init_sizes();
        total += p->ws_bytes();
        b64sum += (double)p->b64_;
    }
    poll_ = pr_[0]->poll_;
    {
        size_t fr = 0, tot = 0;
        SGN_HIP(hipMemGetInfo(&fr, &tot));
        double held = 0.0;
        for (auto &kv : ctx_->basis_pools) held += (double)kv.first * kv.second.size();
        pools_.budget = o_.basis_slots > 0 ? (double)o_.basis_slots * b64sum : 0.5 * ((double)fr + held);
    }
    char *a = static_cast<char *>(ctx_->ensure_arena(total));
    for (size_t k = 0; k < pr_.size(); ++k) {
        pr_[k]->setup(a, st ? st + k : nullptr);
        a += pr_[k]->ws_bytes();
    }
    int active = 0;
    for (auto &p : pr_) active += p->done_ ? 0 : 1;
    const int np = (int)pr_.size();
    {
        std::vector<BsState *> sp(np);
        for (int k = 0; k < np; ++k) sp[k] = pr_[k]->S_;
        dsptr_ = std::make_unique<DeviceScratch>(sizeof(BsState *) * np);
        dheads_ = std::make_unique<DeviceScratch>((sizeof(BsHead) + sizeof(int)) * np);
        dru_ = std::make_unique<DeviceScratch>(2 * sizeof(z64) * np);
        SGN_HIP(hipMemcpy(dsptr_->p, sp.data(), sizeof(BsState *) * np, hipMemcpyHostToDevice));
        SGN_HIP(hipHostMalloc(reinterpret_cast<void **>(&hpin_), (sizeof(BsHead) + sizeof(int)) * np));
        SGN_HIP(hipHostMalloc(reinterpret_cast<void **>(&hru_), 2 * sizeof(z64) * np));
    }
    BsState *const *dsp = static_cast<BsState *const *>(dsptr_->p);
    BsHead *dh = static_cast<BsHead *>(dheads_->p), *hh = reinterpret_cast<BsHead *>(hpin_);
    int *hmask = reinterpret_cast<int *>(hh + np);
    const int *dmask = reinterpret_cast<const int *>(dh + np);
    z64 *dru = static_cast<z64 *>(dru_->p);
    bool dirty = true;
    int finished_since = 0;
    std::vector<BsHead> heads(pr_.size());
    std::vector<int> rus;
    while (active > 0) {
        for (auto &p : pr_)
            if (!p->done_) p->ensure_slots(p->launched_ + poll_);
        if (dirty) {
            rebuild();
            dirty = false;
            finished_since = 0;
        }
        iterate(poll_);
        hipLaunchKernelGGL(bs_gather_heads, dim3(np), dim3(64), 0, s_, dsp, dh);
        SGN_HIP(hipGetLastError());
        SGN_HIP(hipMemcpyAsync(hh, dh, sizeof(BsHead) * np, hipMemcpyDeviceToHost, s_));
        SGN_HIP(hipStreamSynchronize(s_));
        // completions, breakdowns and precision switches take the single-problem path (it writes
        // its head back itself); the reliable updates of all problems go to the device together
        rus.clear();
        for (int k = 0; k < np; ++k) {
            BsStored &p = *pr_[k];
            if (p.done_) continue;
            heads[k] = hh[k];
            const BsHead &h = heads[k];
            const int phase = p.phase_;
            if (h.breakdown || h.done || h.want_phase) {
                if (p.poll(heads[k])) {
                    --active;
                    ++finished_since;
                } else if (p.phase_ != phase) {
                    dirty = true;
                }
            } else if (h.reliable) {
                p.reliable_update_async(h.iter, dru + 2 * k);
                rus.push_back(k);
            } else {
                p.head_ = h;
            }
        }
        if (!rus.empty()) {
            SGN_HIP(hipMemcpyAsync(hru_, dru, 2 * sizeof(z64) * np, hipMemcpyDeviceToHost, s_));
            SGN_HIP(hipStreamSynchronize(s_));
            for (int k = 0; k < np; ++k) hmask[k] = 0;
            for (int k : rus) {
                pr_[k]->reliable_update_finish(heads[k], hru_[2 * k], hru_[2 * k + 1].r);
                hh[k] = heads[k];
                hmask[k] = 1;
            }
            // one copy back and a scatter; the next chunk's launches follow in stream order
            SGN_HIP(hipMemcpyAsync(dh, hh, (sizeof(BsHead) + sizeof(int)) * np, hipMemcpyHostToDevice, s_));
            hipLaunchKernelGGL(bs_scatter_heads, dim3(np), dim3(64), 0, s_, dsp, (const BsHead *)dh, dmask);
            SGN_HIP(hipGetLastError());
        }
        // finished problems only idle in the launches (their kernels see the done flag); drop
        // them once they are a quarter of the launch
        int launched = 0;
        for (auto &g : group_) launched += (int)g.size();
        if (active > 0 && 4 * finished_since >= launched) dirty = true;
    }
    drop_graph();
    sgn_status result = SGN_OK;
    for (size_t k = 0; k < pr_.size(); ++k) {
        if (pr_[k]->ynorm_ == 0.0) continue;  // x = x_P was written by setup
        const sgn_status sk = pr_[k]->finish(st ? st + k : nullptr);
        if (sk != SGN_OK && result == SGN_OK) result = sk;
    }
    return result;
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
        SGN_REQUIRE(o->prec == SGN_PREC_F64 || o->prec == SGN_PREC_F32 || o->prec == SGN_PREC_F32_H16,
                    "multishift_bicgstab: unknown precision");
        SGN_REQUIRE(o->maxiter >= 0 && o->maxiter <= 100000, "multishift_bicgstab: maxiter out of range");
        if (o->basis_slots >= 0 && nprob > 1) {  // stored-basis problems in lockstep
            BsBatch batch(pb, nprob, *rf, *o, static_cast<hipStream_t>(stream));
            result = batch.run(st);
            return;
        }
        for (int k = 0; k < nprob; ++k) {
            const hipStream_t s = static_cast<hipStream_t>(stream);
            sgn_status sk;
            if (o->basis_slots < 0) {
                SGN_REQUIRE(o->prec == SGN_PREC_F64, "multishift_bicgstab: the per-shift form is FP64 only");
                sk = solve_explicit(pb[k], *rf, *o, st ? st + k : nullptr, s);
            } else {
                SGN_REQUIRE(pb[k].lat && pb[k].b && pb[k].x, "multishift_bicgstab: null problem field");
                SGN_REQUIRE(std::isfinite(pb[k].mu), "multishift_bicgstab: mu not finite");
                BsStored solver(pb[k], *rf, *o, s);
                sk = solver.run(st ? st + k : nullptr);
            }
            if (sk != SGN_OK && result == SGN_OK) result = sk;
        }
    });
    return g != SGN_OK ? g : result;
}
