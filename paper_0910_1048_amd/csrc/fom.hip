// Restarted Arnoldi methods for the Neuberger rational function (section
// "Restarted Arnoldi with rational functions"): FOM-LR(m, k) with the collinear
// restart of Eq. (collinearity), and GMRES-LR(m, k) (Algorithm "Restarted
// GMRES-LR", after Frommer and Glassner).
//
// Shifted systems (A' - sigma_i) x_i = y with A' = c^2 H_W(mu)^2, y = c H_W (I-P) b.
// One cycle: k Arnoldi steps on A' from v_1 = r/beta (classical Gram-Schmidt
// applied twice; the Hessenberg columns stay on the device), then on the host
// the small problems of the cycle, x += V_k sum_i omega_i y_i on the device and
// the projection step.
//   FOM:   y_i = beta rho_i (H_k - sigma_i)^{-1} e_1 (Hessenberg LU, O(k^2) each),
//          rho_i <- -h_{k+1,k} e_k^T y_i, r = (I-P) v_{k+1}.
//   GMRES: the seed (shift of smallest modulus) minimises ||beta e_1 - (Hh - sigma_1 Ih) y||
//          (Givens rotations), z = beta e_1 - (Hh - sigma_1 Ih) y_1 is its new residual in
//          the basis V_{k+1}; every other shift solves [Hh - sigma_i Ih | z][y_i; rho_i] =
//          rho_i beta e_1 (bordered Hessenberg LU); r = V_{k+1} z, beta = ||r||,
//          v_1 = (I-P) r / beta.
// Converged when every shifted residual |rho_i| beta <= tol ||y|| (rho = 1 for the seed).
#include <chrono>
#include <complex>
#include <vector>

#include "field_io.h"
#include "vec.h"

namespace sgn {

namespace {

using zc = std::complex<double>;

// H[:, j] = a + b (device, j+1 entries); then hsub = ||w|| and its inverse for the scaling
// Arnoldi column of step j (nj = j + 1 basis vectors): hcol = (2 I - G) h1, with h1 = V^H w and
// G = V^H V (Hermitian; column l of G holds v_i^H v_l for i <= l).  This is classical Gram-Schmidt
// with one reorthogonalisation, whose second-pass dots V^H (w - V h1) = h1 - G h1 come from the
// Gram matrix rather than from a second pass over the basis.
__global__ void fom_gram_kernel(const z64 *G, int ld, int nj, const z64 *h1, z64 *hcol)
{
    for (int i = threadIdx.x; i < nj; i += blockDim.x) {
        z64 acc = {0.0, 0.0};
        for (int l = 0; l < nj; ++l) {
            const z64 g = l >= i ? G[(size_t)l * ld + i] : conj(G[(size_t)i * ld + l]);
            acc = acc + g * h1[l];
        }
        hcol[i] = z64{2.0 * h1[i].r - acc.r, 2.0 * h1[i].i - acc.i};
    }
}

__global__ void fom_norm_kernel(const z64 *partials, int nb, z64 *hsub, z64 *inv)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[i].r;
    __shared__ double lds[4];
    double v[1] = {acc};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) {
        const double h = sqrt(v[0]);
        *hsub = {h, 0.0};
        *inv = {h > 0.0 ? 1.0 / h : 0.0, 0.0};
    }
}

template <typename T>
__device__ __forceinline__ T scaled(T t, double s);
template <> __device__ __forceinline__ double2 scaled<double2>(double2 t, double s) { return make_double2(s * t.x, s * t.y); }
template <> __device__ __forceinline__ float2 scaled<float2>(float2 t, double s)
{
    return make_float2((float)(s * t.x), (float)(s * t.y));
}

// v = w * (*inv)  (inv on the device) or v = w * a
template <typename T>
__global__ void fom_scale_kernel(const T *w, const z64 *inv, double a, T *v, int64_t n)
{
    const double s = inv ? inv->r : a;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        v[e] = scaled<T>(w[e], s);
}

// x[e] += sum_j c_j V_j, V_j FP32 in the [6][S] float4 layout (component c of
// site st at float2 entry 2 ((c/2) S + st) + c%2), x FP64 in the [12][S] layout
__global__ void fom_lift32_kernel(const float2 *basis, int Sst, int k, const z64 *c, double2 *x)
{
    const int64_t n = (int64_t)12 * Sst;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int comp = (int)(e / Sst), st = (int)(e - (int64_t)comp * Sst);
        const int64_t e32 = 2 * ((int64_t)(comp >> 1) * Sst + st) + (comp & 1);
        double2 xv = x[e];
        z64 acc = {xv.x, xv.y};
        for (int j = 0; j < k; ++j) {
            const float2 v = basis[(int64_t)j * n + e32];
            acc = acc + c[j] * z64{(double)v.x, (double)v.y};
        }
        x[e] = make_double2(acc.r, acc.i);
    }
}

// x[e] += sum_j c_j V_j[e]
__global__ void fom_lift_kernel(const double2 *basis, int64_t n, int k, const z64 *c, double2 *x)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double2 xv = x[e];
        z64 acc = {xv.x, xv.y};
        for (int j = 0; j < k; ++j) {
            const double2 v = basis[(int64_t)j * n + e];
            acc = acc + c[j] * z64{v.x, v.y};
        }
        x[e] = make_double2(acc.r, acc.i);
    }
}

// out[e] = sum_j c_j V_j[e]  (FP64 sums; the basis and out in one layout and precision)
template <typename T>
__global__ void fom_comb_kernel(const T *basis, int64_t n, int k, const z64 *c, T *out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        z64 acc = {0.0, 0.0};
        for (int j = 0; j < k; ++j) {
            const T v = basis[(int64_t)j * n + e];
            acc = acc + c[j] * z64{(double)v.x, (double)v.y};
        }
        T o;
        o.x = acc.r;
        o.y = acc.i;
        out[e] = o;
    }
}

// Solve (H - sigma I) y = rhs e_1 for a k x k upper Hessenberg H (column-major
// hc[j*(kmax+1) + i] = H(i,j)), Gaussian elimination with partial pivoting.
bool hessenberg_solve(const std::vector<zc> &hc, int ld, int k, double sigma, zc rhs, std::vector<zc> &y)
{
    std::vector<zc> A((size_t)k * k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i) A[(size_t)i * k + j] = (i <= j + 1) ? hc[(size_t)j * ld + i] : zc(0, 0);
    for (int i = 0; i < k; ++i) A[(size_t)i * k + i] -= sigma;
    std::vector<zc> b(k, zc(0, 0));
    b[0] = rhs;
    for (int i = 0; i + 1 < k; ++i) {  // eliminate the subdiagonal entry of column i
        zc *ri = &A[(size_t)i * k], *rn = &A[(size_t)(i + 1) * k];
        if (std::abs(rn[i]) > std::abs(ri[i])) {
            for (int j = i; j < k; ++j) std::swap(ri[j], rn[j]);
            std::swap(b[i], b[i + 1]);
        }
        if (ri[i] == zc(0, 0)) return false;
        const zc f = rn[i] / ri[i];
        for (int j = i; j < k; ++j) rn[j] -= f * ri[j];
        b[i + 1] -= f * b[i];
    }
    y.assign(k, zc(0, 0));
    for (int i = k - 1; i >= 0; --i) {
        zc acc = b[i];
        for (int j = i + 1; j < k; ++j) acc -= A[(size_t)i * k + j] * y[j];
        if (A[(size_t)i * k + i] == zc(0, 0)) return false;
        y[i] = acc / A[(size_t)i * k + i];
    }
    return true;
}

// Seed of a GMRES cycle: y minimises ||rhs e_1 - (Hh - sigma Ih) y|| for the (k+1) x k
// upper Hessenberg Hh (Givens rotations with real cosines); z = rhs e_1 - (Hh - sigma Ih) y,
// the new residual in the basis V_{k+1}.
bool hessenberg_lsq(const std::vector<zc> &hc, int ld, int k, double sigma, zc rhs, std::vector<zc> &y,
                    std::vector<zc> &z)
{
    auto hs = [&](int i, int j) {  // (Hh - sigma Ih)(i, j)
        zc h = (i <= j + 1) ? hc[(size_t)j * ld + i] : zc(0, 0);
        return i == j ? h - sigma : h;
    };
    std::vector<zc> A((size_t)(k + 1) * k);
    for (int i = 0; i <= k; ++i)
        for (int j = 0; j < k; ++j) A[(size_t)i * k + j] = hs(i, j);
    std::vector<zc> g(k + 1, zc(0, 0));
    g[0] = rhs;
    for (int i = 0; i < k; ++i) {  // rotate rows i, i+1 so that A(i+1, i) = 0
        const zc a = A[(size_t)i * k + i], bb = A[(size_t)(i + 1) * k + i];
        const double aa = std::abs(a), ab = std::abs(bb), t = std::hypot(aa, ab);
        if (t == 0.0) return false;
        const double cs = aa / t;
        const zc sn = aa > 0.0 ? (a / aa) * std::conj(bb) / t : std::conj(bb) / ab;
        for (int j = i; j < k; ++j) {
            const zc u = A[(size_t)i * k + j], v = A[(size_t)(i + 1) * k + j];
            A[(size_t)i * k + j] = cs * u + sn * v;
            A[(size_t)(i + 1) * k + j] = -std::conj(sn) * u + cs * v;
        }
        const zc u = g[i], v = g[i + 1];
        g[i] = cs * u + sn * v;
        g[i + 1] = -std::conj(sn) * u + cs * v;
    }
    y.assign(k, zc(0, 0));
    for (int i = k - 1; i >= 0; --i) {
        zc acc = g[i];
        for (int j = i + 1; j < k; ++j) acc -= A[(size_t)i * k + j] * y[j];
        y[i] = acc / A[(size_t)i * k + i];
    }
    z.assign(k + 1, zc(0, 0));
    z[0] = rhs;
    for (int i = 0; i <= k; ++i)
        for (int j = std::max(i - 1, 0); j < k; ++j) z[i] -= hs(i, j) * y[j];
    return true;
}

// [Hh - sigma Ih | z] [y; rho] = rhs e_1, a (k+1) x (k+1) system whose first k columns
// are upper Hessenberg and whose last column is z; Gaussian elimination with
// partial pivoting between adjacent rows (O(k^2)).
bool bordered_solve(const std::vector<zc> &hc, int ld, int k, double sigma, const std::vector<zc> &z, zc rhs,
                    std::vector<zc> &y, zc &rho)
{
    const int m = k + 1;
    std::vector<zc> A((size_t)m * m, zc(0, 0));
    for (int j = 0; j < k; ++j) {
        for (int i = 0; i <= std::min(j + 1, k); ++i) A[(size_t)i * m + j] = hc[(size_t)j * ld + i];
        A[(size_t)j * m + j] -= sigma;
    }
    for (int i = 0; i < m; ++i) A[(size_t)i * m + k] = z[i];
    std::vector<zc> b(m, zc(0, 0));
    b[0] = rhs;
    for (int i = 0; i < k; ++i) {
        zc *ri = &A[(size_t)i * m], *rn = &A[(size_t)(i + 1) * m];
        if (std::abs(rn[i]) > std::abs(ri[i])) {
            for (int j = i; j < m; ++j) std::swap(ri[j], rn[j]);
            std::swap(b[i], b[i + 1]);
        }
        if (ri[i] == zc(0, 0)) return false;
        const zc f = rn[i] / ri[i];
        for (int j = i; j < m; ++j) rn[j] -= f * ri[j];
        b[i + 1] -= f * b[i];
    }
    std::vector<zc> u(m);
    for (int i = m - 1; i >= 0; --i) {
        zc acc = b[i];
        for (int j = i + 1; j < m; ++j) acc -= A[(size_t)i * m + j] * u[j];
        if (A[(size_t)i * m + i] == zc(0, 0)) return false;
        u[i] = acc / A[(size_t)i * m + i];
    }
    y.assign(u.begin(), u.begin() + k);
    rho = u[k];
    return true;
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

}  // namespace sgn

using namespace sgn;

namespace {

// One restarted Arnoldi driver for both methods; they differ only in the small
// problems solved on the host after each cycle and in the restart vector.
sgn_status restarted_arnoldi(sgn_lattice l, double mu, const void *b, void *x, const sgn_rational *rf,
                             const sgn_deflation *defl, const sgn_arnoldi_opts *o, sgn_stats *st, void *stream,
                             bool gmres)
{
    const std::string who = gmres ? "sign_gmres_rational" : "sign_arnoldi_rational";
    sgn_status result = SGN_OK;
    sgn_status g = guard([&] {
        const auto t_start = std::chrono::steady_clock::now();
        SGN_REQUIRE(l && b && x && rf && o, who + ": null argument");
        SGN_REQUIRE(o->kmax >= 1, who + ": kmax must be >= 1");
        SGN_REQUIRE(o->tol > 0 && o->tol < 1, who + ": tol must be in (0, 1)");
        SGN_REQUIRE(rf->s >= 1 && rf->s <= SGN_MAX_POLES && rf->c > 0, who + ": bad rational function");
        SGN_REQUIRE(o->prec == SGN_PREC_F64 || o->prec == SGN_PREC_F32 || o->prec == SGN_PREC_F32_H16,
                    who + ": unknown precision");
        SGN_REQUIRE(std::isfinite(mu), who + ": mu not finite");
        Lattice &lat = *as_lattice(l);
        Context &ctx = *lat.ctx;
        SGN_HIP(hipSetDevice(ctx.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int k = o->kmax, ns = rf->s;
        // internal vectors: n = 12 S entries (padded stride); canonical: nc = 12 V
        const int64_t V = lat.V, n = 12 * lat.S, nc = 12 * V;
        const size_t b64 = (size_t)n * 16, b32 = (size_t)n * 8, c64 = (size_t)nc * 16;
        const bool mixed = o->prec != SGN_PREC_F64;
        const double theta32 = o->theta32 > 0 ? o->theta32 : 1e-3, theta16 = o->theta16 > 0 ? o->theta16 : 1e-6;
        const int ld = k + 1;
        const double c2 = rf->c * rf->c;
        if (st) {
            *st = sgn_stats{};
            st->nshift = ns;
        }
        // workspace: basis V_{k+1}, w, t, x_int, canonical r (from the arena)
        const size_t hbytes = sizeof(z64) * ((size_t)ld * k + 3 * (size_t)ld + 4 + (size_t)ld * ld);
        char *arena = static_cast<char *>(ctx.ensure_arena((size_t)(k + 1) * b64 + 3 * b64 + c64 + hbytes));
        char *Vb = arena;
        char *w = Vb + (size_t)(k + 1) * b64, *t = w + b64, *xi = t + b64, *rcan = xi + b64;
        z64 *Hd = reinterpret_cast<z64 *>(rcan + c64);  // column-major (k+1) x k
        z64 *h1 = Hd + (size_t)ld * k, *cd = h1 + ld, *scal = cd + ld;  // scal: hsub, inv
        z64 *zd = scal + 4;  // GMRES: the seed's residual z in the basis V_{k+1} (ld entries)
        z64 *Gd = zd + ld;   // Gram matrix V^H V of the cycle's basis, column-major ld x ld (upper triangle)
        bool lo = false;                   // this cycle runs in FP32 (basis slots of b32 bytes)
        sgn_prec sp = SGN_PREC_F64;        // stencil precision of this cycle
        auto Vj = [&](int j) { return Vb + (size_t)j * (lo ? b32 : b64); };

        deflation_prologue(ctx, defl, nc, b, x, rcan, nullptr, s);
        OpSpec opA;
        opA.mu = mu;
        // y = c A r  -> V_0 (unnormalised for now)
        pack_spinor(lat, rcan, t, SGN_PREC_F64, s);
        {
            Epilogue ep;
            ep.a = rf->c;
            dslash_launch(lat, SGN_PREC_F64, opA, t, Vj(0), ep, s);
        }
        const double ynorm = norm_sync(ctx, Vj(0), n, false, s);
        SGN_REQUIRE(std::isfinite(ynorm), who + ": b contains NaN or Inf");
        if (ynorm == 0.0) return;
        SGN_HIP(hipMemsetAsync(xi, 0, b64, s));
        double beta = ynorm;
        scale64({1.0 / beta, 0.0}, Vj(0), Vj(0), n, s);
        std::vector<zc> rho(ns, zc(1, 0));
        std::vector<zc> Hh((size_t)ld * k), y, z, comb(k);
        int seed = 0;  // GMRES: the shift of smallest modulus runs true restarted GMRES
        for (int i = 1; i < ns; ++i)
            if (std::abs(rf->sigma[i]) < std::abs(rf->sigma[seed])) seed = i;
        const int nvb = vec_blocks(n);
        // partials for the widest reduction of a step (two dots per basis vector), sized once
        z64 *part = static_cast<z64 *>(
            ctx.ensure_partials(sizeof(z64) * std::max<size_t>(2 * (size_t)ld * kGramBlocks, (size_t)nvb)));
        const int max_cycles = o->max_restarts > 0 ? o->max_restarts : 1000;
        int cycles = 0, matvecs = 1, steps = 0;
        double small_ms = 0.0;
        const auto t_kry = std::chrono::steady_clock::now();
        bool converged = false;
        double worst_prev = 1.0;  // largest relative shifted residual after the last cycle
        int lo_cycles = 0;
        for (;;) {
            // precision of this cycle: FP32 once every shifted residual is below theta32 (then for good)
            if (mixed && !lo && worst_prev <= theta32) {
                convert_64_to_32(Vb, t, lat.S, s);  // the start vector v_1 moves to the FP32 basis
                SGN_HIP(hipMemcpyAsync(Vb, t, b32, hipMemcpyDeviceToDevice, s));
                lo = true;
                sp = SGN_PREC_F32;
            }
            if (lo && o->prec == SGN_PREC_F32_H16 && worst_prev <= theta16) sp = SGN_PREC_F32_H16;
            lo_cycles += lo ? 1 : 0;
            int kk = k;
            for (int j = 0; j < k; ++j) {
                // w = A' v_j
                dslash_launch(lat, sp, opA, Vj(j), t, Epilogue{}, s);
                Epilogue ep;
                ep.a = c2;
                dslash_launch(lat, sp, opA, t, w, ep, s);
                matvecs += 2;
                // classical Gram-Schmidt with one reorthogonalisation in two passes over the basis
                // (FP64 sums also for an FP32 basis): h1 = V^H w together with the Gram column
                // V^H v_j, the column h = (2 I - G) h1, then w -= V h with the partials of ||w||^2
                gram_dots(Vb, j + 1, w, Vj(j), n, h1, Gd + (size_t)j * ld, ctx, s, lo);
                hipLaunchKernelGGL(fom_gram_kernel, dim3(1), dim3(64), 0, s, (const z64 *)Gd, ld, j + 1,
                                   (const z64 *)h1, Hd + (size_t)j * ld);
                const int nb = combine_norm(w, Vb, j + 1, Hd + (size_t)j * ld, n, part, s, lo);
                hipLaunchKernelGGL(fom_norm_kernel, dim3(1), dim3(256), 0, s, part, nb, Hd + (size_t)j * ld + j + 1,
                                   scal + 1);
                if (lo)
                    hipLaunchKernelGGL(fom_scale_kernel<float2>, dim3(nvb), dim3(256), 0, s, (const float2 *)w,
                                       (const z64 *)(scal + 1), 0.0, (float2 *)Vj(j + 1), n);
                else
                    hipLaunchKernelGGL(fom_scale_kernel<double2>, dim3(nvb), dim3(256), 0, s, (const double2 *)w,
                                       (const z64 *)(scal + 1), 0.0, (double2 *)Vj(j + 1), n);
                SGN_HIP(hipGetLastError());
                ++steps;
            }
            // host: shifted Hessenberg systems of this cycle
            SGN_HIP(hipMemcpyAsync(Hh.data(), Hd, sizeof(z64) * (size_t)ld * k, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipStreamSynchronize(s));
            bool exact = false;  // invariant subspace: the cycle's space holds every solution
            for (int j = 0; j < (gmres ? k : k - 1); ++j)
                if (std::abs(Hh[(size_t)j * ld + j + 1]) == 0.0) {
                    kk = j + 1;
                    exact = true;
                    break;
                }
            const auto t0 = std::chrono::steady_clock::now();
            std::fill(comb.begin(), comb.end(), zc(0, 0));
            if (!gmres || exact) {
                const zc hnext = Hh[(size_t)(kk - 1) * ld + kk];
                for (int i = 0; i < ns; ++i) {
                    if (!hessenberg_solve(Hh, ld, kk, rf->sigma[i], beta * rho[i], y))
                        throw Failure{SGN_ERR_BREAKDOWN, "singular shifted Hessenberg system"};
                    for (int j = 0; j < kk; ++j) comb[j] += rf->omega[i] * y[j];
                    rho[i] = exact ? zc(0, 0) : -hnext * y[kk - 1];
                }
            } else {
                if (!hessenberg_lsq(Hh, ld, k, rf->sigma[seed], beta, y, z))
                    throw Failure{SGN_ERR_BREAKDOWN, "rank-deficient seed least-squares problem"};
                for (int j = 0; j < k; ++j) comb[j] += rf->omega[seed] * y[j];
                for (int i = 0; i < ns; ++i) {
                    if (i == seed) continue;
                    zc ri;
                    if (!bordered_solve(Hh, ld, k, rf->sigma[i], z, beta * rho[i], y, ri))
                        throw Failure{SGN_ERR_BREAKDOWN, "singular collinearity system"};
                    for (int j = 0; j < k; ++j) comb[j] += rf->omega[i] * y[j];
                    rho[i] = ri;
                }
                rho[seed] = zc(1, 0);
            }
            small_ms += ms_since(t0);
            SGN_HIP(hipMemcpyAsync(cd, comb.data(), sizeof(z64) * kk, hipMemcpyHostToDevice, s));
            if (lo)
                hipLaunchKernelGGL(fom_lift32_kernel, dim3(nvb), dim3(256), 0, s, (const float2 *)Vb, (int)lat.S, kk,
                                   cd, (double2 *)xi);
            else
                hipLaunchKernelGGL(fom_lift_kernel, dim3(nvb), dim3(256), 0, s, (const double2 *)Vb, n, kk, cd,
                                   (double2 *)xi);
            ++cycles;
            const bool project = defl && defl->m > 0;
            double rnorm = 1.0;  // FOM: ||(I-P) v_{k+1}||; GMRES: beta = ||V_{k+1} z||
            if (gmres && !exact) {
                // r = V_{k+1} z in w, beta = ||r||, then v_1 = (I-P) r / beta in V_0
                SGN_HIP(hipMemcpyAsync(zd, z.data(), sizeof(z64) * (size_t)(k + 1), hipMemcpyHostToDevice, s));
                if (lo)
                    hipLaunchKernelGGL(fom_comb_kernel<float2>, dim3(nvb), dim3(256), 0, s, (const float2 *)Vb, n,
                                       k + 1, (const z64 *)zd, (float2 *)w);
                else
                    hipLaunchKernelGGL(fom_comb_kernel<double2>, dim3(nvb), dim3(256), 0, s, (const double2 *)Vb, n,
                                       k + 1, (const z64 *)zd, (double2 *)w);
                SGN_HIP(hipGetLastError());
                rnorm = norm_sync(ctx, w, n, lo, s);
                if (project) {
                    if (lo) {
                        convert_32_to_64(w, t, lat.S, s);
                        unpack_spinor(lat, t, rcan, SGN_PREC_F64, s);
                    } else {
                        unpack_spinor(lat, w, rcan, SGN_PREC_F64, s);
                    }
                    deflation_prologue(ctx, defl, nc, rcan, nullptr, t, nullptr, s, false);
                    if (lo) {
                        pack_spinor(lat, t, w, SGN_PREC_F64, s);
                        convert_64_to_32(w, Vj(0), lat.S, s);
                    } else {
                        pack_spinor(lat, t, Vj(0), SGN_PREC_F64, s);
                    }
                } else if (rnorm > 0.0) {  // scaled straight into V_0 below
                    if (lo)
                        hipLaunchKernelGGL(fom_scale_kernel<float2>, dim3(nvb), dim3(256), 0, s, (const float2 *)w,
                                           (const z64 *)nullptr, 1.0 / rnorm, (float2 *)Vj(0), n);
                    else
                        hipLaunchKernelGGL(fom_scale_kernel<double2>, dim3(nvb), dim3(256), 0, s, (const double2 *)w,
                                           (const z64 *)nullptr, 1.0 / rnorm, (double2 *)Vj(0), n);
                    SGN_HIP(hipGetLastError());
                }
            } else if (project && !exact) {
                // r = (I - P) v_{k+1}  (canonical FP64 round trip for the deflation projection)
                if (lo) {
                    convert_32_to_64(Vj(k), w, lat.S, s);
                    unpack_spinor(lat, w, rcan, SGN_PREC_F64, s);
                } else {
                    unpack_spinor(lat, Vj(k), rcan, SGN_PREC_F64, s);
                }
                deflation_prologue(ctx, defl, nc, rcan, nullptr, t, nullptr, s, false);  // t = (I - P) v (canonical)
                if (lo) {
                    pack_spinor(lat, t, w, SGN_PREC_F64, s);
                    convert_64_to_32(w, Vj(0), lat.S, s);
                } else {
                    pack_spinor(lat, t, Vj(0), SGN_PREC_F64, s);
                }
                rnorm = norm_sync(ctx, Vj(0), n, lo, s);
            } else if (!exact) {
                SGN_HIP(hipMemcpyAsync(Vj(0), Vj(k), lo ? b32 : b64, hipMemcpyDeviceToDevice, s));
            }
            double worst = 0.0;
            for (int i = 0; i < ns; ++i) {
                const double ri = std::abs(rho[i]) * rnorm / ynorm;
                worst = std::max(worst, ri);
                if (st) st->shift_residual[i] = ri;
            }
            if (worst <= o->tol || exact) {
                converged = true;
                break;
            }
            if (cycles >= max_cycles) break;
            worst_prev = worst;
            beta = rnorm;
            if (rnorm != 1.0 && (!gmres || project)) {
                if (lo)
                    hipLaunchKernelGGL(fom_scale_kernel<float2>, dim3(nvb), dim3(256), 0, s, (const float2 *)Vj(0),
                                       (const z64 *)nullptr, 1.0 / rnorm, (float2 *)Vj(0), n);
                else
                    scale64({1.0 / rnorm, 0.0}, Vj(0), Vj(0), n, s);
                SGN_HIP(hipGetLastError());
            }
        }
        // x = x_P + x_int
        unpack_spinor(lat, xi, rcan, SGN_PREC_F64, s);
        axpby64({1.0, 0.0}, rcan, {1.0, 0.0}, x, nc, s);
        SGN_HIP(hipStreamSynchronize(s));
        if (!converged) result = SGN_ERR_NOT_CONVERGED;
        if (st) {
            st->iterations = steps;
            st->restarts = cycles;
            st->reliable_updates = lo_cycles;  // cycles run with the FP32 basis
            st->matvecs = matvecs;
            double worst = 0.0;
            for (int i = 0; i < ns; ++i) worst = std::max(worst, st->shift_residual[i]);
            st->residual = worst;
            st->small_ms = small_ms;
            st->krylov_ms = ms_since(t_kry);
            st->total_ms = ms_since(t_start);
        }
    });
    return g != SGN_OK ? g : result;
}

}  // namespace

extern "C" sgn_status sign_arnoldi_rational(sgn_lattice l, double mu, const void *b, void *x, const sgn_rational *rf,
                                           const sgn_deflation *defl, const sgn_arnoldi_opts *o, sgn_stats *st,
                                           void *stream)
{
    return restarted_arnoldi(l, mu, b, x, rf, defl, o, st, stream, false);
}

extern "C" sgn_status sign_gmres_rational(sgn_lattice l, double mu, const void *b, void *x, const sgn_rational *rf,
                                         const sgn_deflation *defl, const sgn_arnoldi_opts *o, sgn_stats *st,
                                         void *stream)
{
    return restarted_arnoldi(l, mu, b, x, rf, defl, o, st, stream, true);
}
