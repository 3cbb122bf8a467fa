// Critical eigenpairs of H_W(mu) for LR deflation (section "Deflation").
//
// The critical eigenvalues of sign are those closest to the imaginary axis; LR
// deflation needs their right eigenvectors R (H R = R Lambda) and left
// eigenvectors L (L^H H = Lambda L^H) with L^H R = I.  Zero lies inside the
// spectrum of H_W (eigenvalues near both halves of the real axis), where a
// Krylov process converges poorly; for A = H_W^2 the eigenvalues lambda^2 =
// x^2 - y^2 + 2ixy of the critical eigenvalues have the smallest real parts,
// at one end of the spectrum of A.  Hence:
//
//  1. Implicitly restarted Arnoldi with exact shifts on A = H_W(mu)^2: k
//     Arnoldi steps (classical Gram-Schmidt twice, FP64 stencil), Ritz values
//     of the k x k Hessenberg matrix, the k - p of largest real part used as
//     shifts of implicit QR steps, the basis compressed to p + 1 vectors and
//     extended again, until the m + 2 wanted Ritz pairs of smallest real part
//     have residual |h_{k+1,k} e_k^T y| <= tol |theta|.
//  2. The same on H_W(-mu) = H_W(mu)^H (left eigenvectors are right
//     eigenvectors of the adjoint, for conj(lambda)).
//  3. Rayleigh-Ritz with H_W itself on the converged wanted Ritz vectors of each
//     side; Ritz pairs with a large residual (a vector mixing eigenvectors of
//     lambda and -lambda' has a Rayleigh quotient near 0) are dropped; the m Ritz
//     values of smallest |Re| selected and their span orthonormalised: Q_R
//     (right), Q_L (left), n x m each.
//  4. Oblique projection: M = Q_L^H Q_R, C = Q_L^H H Q_R, M^{-1} C = Y Lambda Y^{-1};
//     R = Q_R Y (unit columns), L^H = Y^{-1} M^{-1} Q_L^H.  Then L^H R = I, and
//     on exactly invariant subspaces H R = R Lambda and L^H H = Lambda L^H.
//
// Small dense work (Hessenberg eigenproblems, QR steps, m x m inverses) runs on
// the host in FP64; every vector operation runs on the device.
#include <algorithm>
#include <chrono>
#include <complex>
#include <numeric>
#include <string>
#include <vector>

#include "field_io.h"
#include "small_sign.h"
#include "vec.h"

namespace sgn {

namespace {

using zc = std::complex<double>;

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Deterministic pseudo-random start vector in the internal FP64 layout [12][S]:
// entry (component c, site st < V) from splitmix64 of (seed, c, st), uniform in
// [-1/2, 1/2) per real part; padding sites [V, S) stay zero.
__global__ void eig_fill_kernel(double2 *v, int64_t S, int64_t V, unsigned long long seed)
{
    const int64_t n = 12 * S;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t st = e % S;
        double2 out = make_double2(0.0, 0.0);
        if (st < V) {
            const unsigned long long h1 = splitmix64(seed * 0x100000001B3ull + 2 * (unsigned long long)e);
            const unsigned long long h2 = splitmix64(seed * 0x100000001B3ull + 2 * (unsigned long long)e + 1);
            out.x = (double)(h1 >> 11) * 0x1.0p-53 - 0.5;
            out.y = (double)(h2 >> 11) * 0x1.0p-53 - 0.5;
        }
        v[e] = out;
    }
}

// out_j = sum_i Q[i * nout + j] V_i  for j < nout (vectors of n entries back to back);
// outputs in chunks of 8 per pass over the inputs
constexpr int kCombChunk = 8;
__global__ void eig_combine_kernel(const double2 *V, int64_t n, int kin, const z64 *Q, int nout, double2 *out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        for (int j0 = 0; j0 < nout; j0 += kCombChunk) {
            const int nj = min(kCombChunk, nout - j0);
            z64 acc[kCombChunk];
#pragma unroll
            for (int jj = 0; jj < kCombChunk; ++jj) acc[jj] = {0.0, 0.0};
            for (int i = 0; i < kin; ++i) {
                const double2 v = V[(int64_t)i * n + e];
                const z64 vz = {v.x, v.y};
#pragma unroll
                for (int jj = 0; jj < kCombChunk; ++jj)
                    if (jj < nj) acc[jj] = acc[jj] + Q[(int64_t)i * nout + j0 + jj] * vz;
            }
            for (int jj = 0; jj < nj; ++jj) out[(int64_t)(j0 + jj) * n + e] = make_double2(acc[jj].r, acc[jj].i);
        }
    }
}

// Arnoldi column j on the device: h_i = c1_i + c2_i (the two Gram-Schmidt passes) into column j
// of the Hessenberg matrix hd (column-major, leading dimension ld), beta = ||w|| from the norm
// partials pn[0..nb) (summed in a fixed order), and step[j] = {1 / beta, 0}, or {0, 1} when
// beta <= 1e-13 ||h|| (an invariant subspace: the host restarts from that column).
__global__ void __launch_bounds__(256) eig_hcol_kernel(const z64 *c1, const z64 *c2, int j, int ld, const z64 *pn,
                                                       int nb, z64 *hd, z64 *step)
{
    __shared__ double lds[8];
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v[0] += pn[b].r;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        const z64 h = c1[i] + c2[i];
        hd[(size_t)j * ld + i] = h;
        v[1] += norm2(h);
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        const double beta = sqrt(v[0]);
        const bool ok = beta > 1e-13 * sqrt(v[1]);
        hd[(size_t)j * ld + j + 1] = {ok ? beta : 0.0, 0.0};
        step[j] = ok ? z64{1.0 / beta, 0.0} : z64{0.0, 1.0};
    }
}

// v = step->r * w (zero after a breakdown)
__global__ void __launch_bounds__(256) eig_scale_kernel(const double2 *w, double2 *v, int64_t n, const z64 *step)
{
    const double a = step->r;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 x = w[e];
        v[e] = make_double2(a * x.x, a * x.y);
    }
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// inverse of a small complex matrix (row-major), Gauss-Jordan with partial pivoting
bool small_inverse(int n, const std::vector<zc> &a, std::vector<zc> &inv)
{
    std::vector<zc> A = a;
    inv.assign((size_t)n * n, zc(0, 0));
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(A[(size_t)r * n + c]) > std::abs(A[(size_t)piv * n + c])) piv = r;
        if (A[(size_t)piv * n + c] == zc(0, 0)) return false;
        if (piv != c)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)piv * n + j], A[(size_t)c * n + j]);
                std::swap(inv[(size_t)piv * n + j], inv[(size_t)c * n + j]);
            }
        const zc d = 1.0 / A[(size_t)c * n + c];
        for (int j = 0; j < n; ++j) {
            A[(size_t)c * n + j] *= d;
            inv[(size_t)c * n + j] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const zc f = A[(size_t)r * n + c];
            if (f == zc(0, 0)) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
                inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
            }
        }
    }
    return true;
}

// columns of the k x q row-major matrix Y orthonormalised in place (modified Gram-Schmidt, twice)
void orthonormalise_columns(int k, int q, std::vector<zc> &Y)
{
    for (int j = 0; j < q; ++j) {
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                zc d = 0.0;
                for (int r = 0; r < k; ++r) d += std::conj(Y[(size_t)r * q + i]) * Y[(size_t)r * q + j];
                for (int r = 0; r < k; ++r) Y[(size_t)r * q + j] -= d * Y[(size_t)r * q + i];
            }
        double nr = 0.0;
        for (int r = 0; r < k; ++r) nr += std::norm(Y[(size_t)r * q + j]);
        nr = std::sqrt(nr);
        if (!(nr > 0.0)) throw Failure{SGN_ERR_BREAKDOWN, "eigensolver: dependent Ritz vectors"};
        for (int r = 0; r < k; ++r) Y[(size_t)r * q + j] /= nr;
    }
}

struct EigSolver {
    Lattice &lat;
    Context &ctx;
    hipStream_t s;
    int m, p, k;
    double tol;
    int max_restarts;
    unsigned long long seed;
    int64_t n;     // 12 S entries per internal vector
    size_t b64;    // bytes per internal vector
    char *Va, *Vb;  // two bases of k + 1 vectors
    char *w, *t;
    z64 *cd;        // device coefficients (k + 1) * (k + 1)
    z64 *c1, *c2;   // device Gram-Schmidt coefficients (k + 1 each)
    z64 *hd;        // device Hessenberg matrix of extend, (k + 1) x k column-major
    z64 *pn;        // device norm partials (kMaxBlocks)
    z64 *dstep;     // device per column: {1 / beta, breakdown}

    int nvb;
    // statistics
    int steps = 0, matvecs = 0, restarts = 0;
    double small_ms = 0.0;

    void fill_random(void *v, unsigned long long sd)
    {
        hipLaunchKernelGGL(eig_fill_kernel, dim3(nvb), dim3(256), 0, s, (double2 *)v, (int64_t)lat.S, (int64_t)lat.V,
                           sd);
        SGN_HIP(hipGetLastError());
    }

    void combine(const void *V, int kin, const std::vector<zc> &Q, int nout, void *out)
    {
        SGN_HIP(hipMemcpyAsync(cd, Q.data(), sizeof(z64) * (size_t)kin * nout, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(eig_combine_kernel, dim3(nvb), dim3(256), 0, s, (const double2 *)V, n, kin,
                           (const z64 *)cd, nout, (double2 *)out);
        SGN_HIP(hipGetLastError());
        SGN_HIP(hipStreamSynchronize(s));  // cd is reused by the next call
    }

    // w -= V_0..V_{j} (V_i^H w), twice; returns the summed coefficients
    void cgs2(const char *V, int nv, void *x, std::vector<zc> &h)
    {
        deflate_dots(V, nv, x, n, c1, ctx, s);
        deflate_combine(x, {1.0, 0.0}, {-1.0, 0.0}, V, nv, c1, nullptr, n, s);
        deflate_dots(V, nv, x, n, c2, ctx, s);
        deflate_combine(x, {1.0, 0.0}, {-1.0, 0.0}, V, nv, c2, nullptr, n, s);
        std::vector<zc> a(nv), b(nv);
        SGN_HIP(hipMemcpyAsync(a.data(), c1, sizeof(z64) * nv, hipMemcpyDeviceToHost, s));
        SGN_HIP(hipMemcpyAsync(b.data(), c2, sizeof(z64) * nv, hipMemcpyDeviceToHost, s));
        SGN_HIP(hipStreamSynchronize(s));
        h.resize(nv);
        for (int i = 0; i < nv; ++i) h[i] = a[i] + b[i];
    }

    char *vec(char *V, int i) const { return V + (size_t)i * b64; }

    // Arnoldi steps j0 .. k-1 on A = H(mu)^2; H column-major, ld = k + 1.  The steps run without
    // host synchronisation: the Gram-Schmidt coefficients, the Hessenberg column, the norm and the
    // normalisation stay on the device, and H and the breakdown flags are read once at the end.
    void extend(char *V, const OpSpec &op, std::vector<zc> &H, int j0)
    {
        const int ld = k + 1;
        std::vector<zc> hcol((size_t)ld * k);
        std::vector<z64> stp(k);
        // the partials of the largest basis, so that the buffer does not grow (and wait for the
        // device) between the steps
        ctx.ensure_partials(deflate_partials_bytes(ld, n));
        while (j0 < k) {
            for (int j = j0; j < k; ++j) {
                dslash_launch(lat, SGN_PREC_F64, op, vec(V, j), t, Epilogue{}, s);
                dslash_launch(lat, SGN_PREC_F64, op, t, w, Epilogue{}, s);
                deflate_dots(V, j + 1, w, n, c1, ctx, s);
                deflate_combine(w, {1.0, 0.0}, {-1.0, 0.0}, V, j + 1, c1, nullptr, n, s);
                deflate_dots(V, j + 1, w, n, c2, ctx, s);
                deflate_combine(w, {1.0, 0.0}, {-1.0, 0.0}, V, j + 1, c2, nullptr, n, s);
                const int nb = norm2_partials(w, n, false, pn, s);
                hipLaunchKernelGGL(eig_hcol_kernel, dim3(1), dim3(256), 0, s, (const z64 *)c1, (const z64 *)c2, j, ld,
                                   (const z64 *)pn, nb, hd, dstep);
                hipLaunchKernelGGL(eig_scale_kernel, dim3(nvb), dim3(256), 0, s, (const double2 *)w,
                                   (double2 *)vec(V, j + 1), n, (const z64 *)(dstep + j));
                SGN_HIP(hipGetLastError());
            }
            matvecs += 2 * (k - j0);
            steps += k - j0;
            SGN_HIP(hipMemcpyAsync(hcol.data(), hd, sizeof(z64) * hcol.size(), hipMemcpyDeviceToHost, s));
            SGN_HIP(hipMemcpyAsync(stp.data(), dstep, sizeof(z64) * k, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipStreamSynchronize(s));
            int jb = k;  // the first column whose residual vanished
            for (int j = j0; j < k && jb == k; ++j)
                if (stp[j].i != 0.0) jb = j;
            for (int j = j0; j < std::min(jb + 1, k); ++j)
                for (int i = 0; i <= j + 1; ++i) H[(size_t)j * ld + i] = hcol[(size_t)j * ld + i];
            if (jb == k) break;
            // invariant subspace found at column jb: continue from a fresh vector orthogonal to the
            // basis (the columns after jb are recomputed)
            fill_random(w, seed + 0x1000 + (unsigned long long)steps);
            std::vector<zc> dummy;
            cgs2(V, jb + 1, w, dummy);
            const double r = norm_sync(ctx, w, n, false, s);
            scale64({1.0 / r, 0.0}, w, vec(V, jb + 1), n, s);
            H[(size_t)jb * ld + jb + 1] = 0.0;
            j0 = jb + 1;
        }
    }

    // Implicitly restarted Arnoldi on H(mu_side)^2.  On return V (one of the two
    // bases) holds the k-step Arnoldi basis of the last cycle and Yw (k x q,
    // row-major, orthonormal columns, m + 2 <= q <= p) spans its leading converged
    // wanted Ritz vectors.
    bool iram(double mu_side, unsigned long long sd, char *&V, std::vector<zc> &Yw)
    {
        OpSpec op;
        op.mu = mu_side;
        const int ld = k + 1;
        V = Va;
        char *Vo = Vb;
        fill_random(vec(V, 0), sd);
        const double r0 = norm_sync(ctx, vec(V, 0), n, false, s);
        scale64({1.0 / r0, 0.0}, vec(V, 0), vec(V, 0), n, s);
        std::vector<zc> H((size_t)ld * k, zc(0, 0));
        int j0 = 0;
        const int mc = std::min(p, m + 2);
        bool converged = false;
        std::vector<zc> Hk((size_t)k * k), theta(k), Y((size_t)k * k);
        std::vector<int> order(k);
        for (int cycle = 0;; ++cycle) {
            extend(V, op, H, j0);
            const auto t0 = std::chrono::steady_clock::now();
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j) Hk[(size_t)i * k + j] = (i <= j + 1) ? H[(size_t)j * ld + i] : zc(0, 0);
            if (small_eig(k, Hk.data(), theta.data(), Y.data()) != 0)
                throw Failure{SGN_ERR_BREAKDOWN, "eigensolver: Hessenberg QR did not converge"};
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return theta[a].real() < theta[b].real(); });
            const double hk = std::abs(H[(size_t)(k - 1) * ld + k]);
            converged = true;
            for (int i = 0; i < mc; ++i) {
                const int c = order[i];
                if (hk * std::abs(Y[(size_t)(k - 1) * k + c]) > tol * std::abs(theta[c])) converged = false;
            }
            if (converged || cycle >= max_restarts) {
                // the Rayleigh-Ritz subspace: the leading wanted Ritz vectors that have converged
                // (all p when the iteration stopped unconverged); an unconverged one can mix
                // eigenvectors of lambda and -lambda' and give a spurious Ritz value of H near 0
                int q = p;
                if (converged) {
                    q = mc;
                    while (q < p && hk * std::abs(Y[(size_t)(k - 1) * k + order[q]]) <= tol * std::abs(theta[order[q]]))
                        ++q;
                }
                Yw.assign((size_t)k * q, zc(0, 0));
                for (int r = 0; r < k; ++r)
                    for (int j = 0; j < q; ++j) Yw[(size_t)r * q + j] = Y[(size_t)r * k + order[j]];
                orthonormalise_columns(k, q, Yw);
                small_ms += ms_since(t0);
                return converged;
            }
            ++restarts;
            // implicit QR steps with the k - p unwanted Ritz values as shifts
            std::vector<zc> Q((size_t)k * k, zc(0, 0));
            for (int i = 0; i < k; ++i) Q[(size_t)i * k + i] = 1.0;
            std::vector<double> gc(k);
            std::vector<zc> gs(k);
            for (int u = p; u < k; ++u) {
                const zc sh = theta[order[u]];
                for (int i = 0; i < k; ++i) Hk[(size_t)i * k + i] -= sh;
                for (int i = 0; i + 1 < k; ++i) {  // QR of the shifted Hessenberg matrix
                    const zc x = Hk[(size_t)i * k + i], y = Hk[(size_t)(i + 1) * k + i];
                    const double ax = std::abs(x), ay = std::abs(y);
                    double c;
                    zc sn;
                    if (ay == 0.0) {
                        c = 1.0;
                        sn = 0.0;
                    } else if (ax == 0.0) {
                        c = 0.0;
                        sn = std::conj(y) / ay;
                    } else {
                        const double nr = std::hypot(ax, ay);
                        c = ax / nr;
                        sn = (x / ax) * std::conj(y) / nr;
                    }
                    gc[i] = c;
                    gs[i] = sn;
                    for (int j = i; j < k; ++j) {
                        const zc t1 = Hk[(size_t)i * k + j], t2 = Hk[(size_t)(i + 1) * k + j];
                        Hk[(size_t)i * k + j] = c * t1 + sn * t2;
                        Hk[(size_t)(i + 1) * k + j] = -std::conj(sn) * t1 + c * t2;
                    }
                }
                for (int i = 0; i + 1 < k; ++i) {  // R Q, and Q accumulates
                    const double c = gc[i];
                    const zc sn = gs[i];
                    for (int r = 0; r <= std::min(i + 1, k - 1); ++r) {
                        const zc t1 = Hk[(size_t)r * k + i], t2 = Hk[(size_t)r * k + i + 1];
                        Hk[(size_t)r * k + i] = t1 * c + t2 * std::conj(sn);
                        Hk[(size_t)r * k + i + 1] = -t1 * sn + t2 * c;
                    }
                    for (int r = 0; r < k; ++r) {
                        const zc t1 = Q[(size_t)r * k + i], t2 = Q[(size_t)r * k + i + 1];
                        Q[(size_t)r * k + i] = t1 * c + t2 * std::conj(sn);
                        Q[(size_t)r * k + i + 1] = -t1 * sn + t2 * c;
                    }
                }
                for (int i = 0; i < k; ++i) Hk[(size_t)i * k + i] += sh;
                for (int i = 2; i < k; ++i)
                    for (int j = 0; j + 1 < i; ++j) Hk[(size_t)i * k + j] = 0.0;
            }
            // compressed basis V_p Q(:, 0..p-1) and residual f = V_k Q(:, p) Hk(p, p-1) + h_{k+1,k} Q(k-1, p-1) v_{k+1}
            std::vector<zc> Qp((size_t)k * p);
            for (int r = 0; r < k; ++r)
                for (int j = 0; j < p; ++j) Qp[(size_t)r * p + j] = Q[(size_t)r * k + j];
            std::vector<zc> fq(k + 1);
            const zc bp = Hk[(size_t)p * k + p - 1];
            for (int r = 0; r < k; ++r) fq[r] = Q[(size_t)r * k + p] * bp;
            fq[k] = H[(size_t)(k - 1) * ld + k] * Q[(size_t)(k - 1) * k + p - 1];
            small_ms += ms_since(t0);
            combine(V, k, Qp, p, Vo);
            combine(V, k + 1, fq, 1, w);
            std::vector<zc> dummy;
            cgs2(Vo, p, w, dummy);  // keep the restarted basis orthonormal to rounding
            const double fn = norm_sync(ctx, w, n, false, s);
            scale64({1.0 / fn, 0.0}, w, vec(Vo, p), n, s);
            std::swap(V, Vo);
            std::fill(H.begin(), H.end(), zc(0, 0));
            for (int j = 0; j < p; ++j)
                for (int i = 0; i <= std::min(j + 1, p - 1); ++i) H[(size_t)j * ld + i] = Hk[(size_t)i * k + j];
            H[(size_t)(p - 1) * ld + p] = fn;
            j0 = p;
        }
    }

    // Rayleigh-Ritz with H(mu_side) on span(V Yw) (q = columns of Yw): Ritz pairs
    // (theta, u = V Yw x) with residual ||H u - theta u||^2 = x^H (HQ^H HQ) x - |theta|^2
    // above kRitzScreen |theta| are dropped as spurious; of the rest, the m of smallest
    // |Re theta| are selected and their span orthonormalised: Z (k x m, row-major)
    // gives that basis as V Z.  theta_rest receives the moduli of the kept, unselected
    // Ritz values.
    static constexpr double kRitzScreen = 1e-4;
    void ritz_select(double mu_side, const char *V, const std::vector<zc> &Yw, char *T, std::vector<zc> &Z,
                     std::vector<double> &theta_rest)
    {
        OpSpec op;
        op.mu = mu_side;
        const int q = (int)(Yw.size() / k);
        char *Qp = T;                        // q vectors: V Yw
        char *HQ = T + (size_t)q * b64;      // q vectors: H V Yw
        combine(V, k, Yw, q, Qp);
        for (int i = 0; i < q; ++i) {
            dslash_launch(lat, SGN_PREC_F64, op, vec(Qp, i), vec(HQ, i), Epilogue{}, s);
            ++matvecs;
        }
        std::vector<zc> G((size_t)q * q), Gh((size_t)q * q), col(q);
        for (int i = 0; i < q; ++i) {
            deflate_dots(Qp, q, vec(HQ, i), n, c1, ctx, s);
            deflate_dots(HQ, q, vec(HQ, i), n, c2, ctx, s);
            SGN_HIP(hipMemcpyAsync(col.data(), c1, sizeof(z64) * q, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipStreamSynchronize(s));
            for (int r = 0; r < q; ++r) G[(size_t)r * q + i] = col[r];
            SGN_HIP(hipMemcpyAsync(col.data(), c2, sizeof(z64) * q, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipStreamSynchronize(s));
            for (int r = 0; r < q; ++r) Gh[(size_t)r * q + i] = col[r];
        }
        std::vector<zc> th(q), X((size_t)q * q);
        if (small_eig(q, G.data(), th.data(), X.data()) != 0)
            throw Failure{SGN_ERR_BREAKDOWN, "eigensolver: Rayleigh-Ritz QR did not converge"};
        std::vector<int> keep;
        for (int j = 0; j < q; ++j) {
            double r2 = 0.0;
            for (int a = 0; a < q; ++a) {
                zc acc = 0.0;
                for (int b = 0; b < q; ++b) acc += Gh[(size_t)a * q + b] * X[(size_t)b * q + j];
                r2 += (std::conj(X[(size_t)a * q + j]) * acc).real();
            }
            r2 -= std::norm(th[j]);
            if (std::sqrt(std::max(r2, 0.0)) <= kRitzScreen * std::abs(th[j])) keep.push_back(j);
        }
        if ((int)keep.size() < m)
            throw Failure{SGN_ERR_NOT_CONVERGED, "eigensolver: " + std::to_string(keep.size()) + " of the " +
                                                     std::to_string(m) + " wanted Ritz pairs accurate (" +
                                                     std::to_string(restarts) + " restarts)"};
        std::stable_sort(keep.begin(), keep.end(),
                         [&](int a, int b) { return std::abs(th[a].real()) < std::abs(th[b].real()); });
        theta_rest.clear();
        for (size_t j = m; j < keep.size(); ++j) theta_rest.push_back(std::abs(th[keep[j]]));
        std::vector<zc> Xs((size_t)q * m);
        for (int r = 0; r < q; ++r)
            for (int j = 0; j < m; ++j) Xs[(size_t)r * m + j] = X[(size_t)r * q + keep[j]];
        orthonormalise_columns(q, m, Xs);
        Z.assign((size_t)k * m, zc(0, 0));  // Yw Xs
        for (int r = 0; r < k; ++r)
            for (int j = 0; j < m; ++j) {
                zc acc = 0.0;
                for (int l = 0; l < q; ++l) acc += Yw[(size_t)r * q + l] * Xs[(size_t)l * m + j];
                Z[(size_t)r * m + j] = acc;
            }
    }
};

}  // namespace

}  // namespace sgn

using namespace sgn;

extern "C" sgn_status sgn_critical_eigenpairs(sgn_lattice l, double mu, const sgn_eig_opts *o, void *Lout,
                                              void *Rout, double *lambda, double *alpha, sgn_stats *st, void *stream)
{
    return guard([&] {
        const auto t_start = std::chrono::steady_clock::now();
        SGN_REQUIRE(l && o && Lout && Rout && lambda, "sgn_critical_eigenpairs: null argument");
        SGN_REQUIRE(std::isfinite(mu), "sgn_critical_eigenpairs: mu not finite");
        Lattice &lat = *as_lattice(l);
        Context &ctx = *lat.ctx;
        SGN_HIP(hipSetDevice(ctx.device));
        const int m = o->m;
        // defaults: a basis large enough for clustered spectra (at 8^4 with m = 4, 24 kept pairs of a
        // 64-vector basis need 86 restarts where 10 of 36 need 545), held below the vector length
        const int64_t nlen = 12 * lat.V;
        const int k = o->kmax > 0 ? o->kmax
                                  : (int)std::min<int64_t>({2 * (m + std::max(20, m)) + 16, 1024, nlen - 1});
        const int p = o->nev > 0 ? o->nev : std::min(m + std::max(20, m), k - 2);
        SGN_REQUIRE(m >= 1, "sgn_critical_eigenpairs: m must be >= 1");
        SGN_REQUIRE(p > m, "sgn_critical_eigenpairs: nev must exceed m");
        SGN_REQUIRE(k >= p + 2 && k <= 1024, "sgn_critical_eigenpairs: kmax must be in [nev + 2, 1024]");
        SGN_REQUIRE((int64_t)k < 12 * lat.V, "sgn_critical_eigenpairs: kmax must be below the vector length");
        SGN_REQUIRE(!(o->tol < 0) && o->tol < 1, "sgn_critical_eigenpairs: tol must be in [0, 1)");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (st) *st = sgn_stats{};
        const int64_t n = 12 * lat.S, nc = 12 * lat.V;
        const size_t b64 = (size_t)n * 16;
        // workspace: 2 bases of k + 1 vectors, w, t, 2p (Ritz block), Q_R, Q_L, H Q_R (m each), coefficients
        const size_t nvec = 2 * (size_t)(k + 1) + 2 + 2 * (size_t)p + 3 * (size_t)m;
        const size_t cbytes =
            sizeof(z64) * ((size_t)(k + 1) * (k + 1) + 2 * (size_t)(k + 1) + (size_t)(k + 1) * k + kMaxBlocks + k);
        char *arena = static_cast<char *>(ctx.ensure_arena(nvec * b64 + cbytes));
        EigSolver E{lat, ctx, s, m, p, k, o->tol > 0 ? o->tol : 1e-10, o->max_restarts > 0 ? o->max_restarts : 1000,
                    (unsigned long long)o->seed, n, b64};
        E.Va = arena;
        E.Vb = E.Va + (size_t)(k + 1) * b64;
        E.w = E.Vb + (size_t)(k + 1) * b64;
        E.t = E.w + b64;
        char *T = E.t + b64;                   // 2p vectors
        char *QR = T + 2 * (size_t)p * b64;    // m
        char *QL = QR + (size_t)m * b64;       // m
        char *HQ = QL + (size_t)m * b64;       // m
        E.cd = reinterpret_cast<z64 *>(HQ + (size_t)m * b64);
        E.c1 = E.cd + (size_t)(k + 1) * (k + 1);
        E.c2 = E.c1 + (k + 1);
        E.hd = E.c2 + (k + 1);
        E.pn = E.hd + (size_t)(k + 1) * k;
        E.dstep = E.pn + kMaxBlocks;
        E.nvb = vec_blocks(n);
        const double mus[2] = {mu, -mu};
        char *Qs[2] = {QR, QL};
        std::vector<double> rest_right;
        bool converged = true;
        // the work done so far, also when a side stops without enough accurate pairs
        auto record = [&](double worst) {
            if (!st) return;
            st->iterations = E.steps;
            st->matvecs = E.matvecs;
            st->restarts = E.restarts;
            st->residual = worst;
            st->small_ms = E.small_ms;
            st->total_ms = ms_since(t_start);
        };
        try {
            for (int side = 0; side < 2; ++side) {
                char *V = nullptr;
                std::vector<zc> Yw, Z;
                std::vector<double> th;
                converged = E.iram(mus[side], E.seed * 2 + side + 1, V, Yw) && converged;
                E.ritz_select(mus[side], V, Yw, T, Z, th);
                E.combine(V, k, Z, m, Qs[side]);
                if (side == 0) rest_right = th;
            }
        } catch (...) {
            record(0.0);
            throw;
        }
        // oblique projection on the pair of invariant subspaces
        OpSpec op;
        op.mu = mu;
        for (int i = 0; i < m; ++i) {
            dslash_launch(lat, SGN_PREC_F64, op, E.vec(QR, i), E.vec(HQ, i), Epilogue{}, s);
            ++E.matvecs;
        }
        std::vector<zc> M((size_t)m * m), C((size_t)m * m), col(m);
        for (int i = 0; i < m; ++i) {
            deflate_dots(QL, m, E.vec(QR, i), n, E.c1, ctx, s);
            deflate_dots(QL, m, E.vec(HQ, i), n, E.c2, ctx, s);
            SGN_HIP(hipMemcpyAsync(col.data(), E.c1, sizeof(z64) * m, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipStreamSynchronize(s));
            for (int r = 0; r < m; ++r) M[(size_t)r * m + i] = col[r];
            SGN_HIP(hipMemcpyAsync(col.data(), E.c2, sizeof(z64) * m, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipStreamSynchronize(s));
            for (int r = 0; r < m; ++r) C[(size_t)r * m + i] = col[r];
        }
        std::vector<zc> Minv, G((size_t)m * m), lam(m), Y((size_t)m * m), Yinv;
        if (!small_inverse(m, M, Minv))
            throw Failure{SGN_ERR_BREAKDOWN, "eigensolver: left and right invariant subspaces do not pair"};
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                zc acc = 0.0;
                for (int l2 = 0; l2 < m; ++l2) acc += Minv[(size_t)i * m + l2] * C[(size_t)l2 * m + j];
                G[(size_t)i * m + j] = acc;
            }
        std::vector<zc> lam0(m), Y0((size_t)m * m);
        if (small_eig(m, G.data(), lam0.data(), Y0.data()) != 0)
            throw Failure{SGN_ERR_BREAKDOWN, "eigensolver: projected QR did not converge"};
        std::vector<int> order(m);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return std::abs(lam0[a].real()) < std::abs(lam0[b].real()); });
        for (int j = 0; j < m; ++j) {
            lam[j] = lam0[order[j]];
            for (int r = 0; r < m; ++r) Y[(size_t)r * m + j] = Y0[(size_t)r * m + order[j]];
        }
        if (!small_inverse(m, Y, Yinv)) throw Failure{SGN_ERR_BREAKDOWN, "eigensolver: defective projected matrix"};
        // L = Q_L W with W = (Y^{-1} M^{-1})^H
        std::vector<zc> W((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                zc acc = 0.0;
                for (int l2 = 0; l2 < m; ++l2) acc += Yinv[(size_t)j * m + l2] * Minv[(size_t)l2 * m + i];
                W[(size_t)i * m + j] = std::conj(acc);
            }
        char *Rint = T, *Lint = T + (size_t)m * b64;  // 2m <= 2p vectors
        E.combine(QR, m, Y, m, Rint);
        E.combine(QL, m, W, m, Lint);
        // residuals ||H r - lambda r|| / ||r||, ||H^H l - conj(lambda) l|| / ||l||
        double worst = 0.0;
        for (int i = 0; i < m; ++i) {
            for (int side = 0; side < 2; ++side) {
                const char *v = E.vec(side == 0 ? Rint : Lint, i);
                OpSpec os;
                os.mu = mus[side];
                Epilogue ep;
                ep.b = side == 0 ? z64{-lam[i].real(), -lam[i].imag()} : z64{-lam[i].real(), lam[i].imag()};
                ep.z = v;
                dslash_launch(lat, SGN_PREC_F64, os, v, E.w, ep, s);
                ++E.matvecs;
                const double rn = norm_sync(ctx, E.w, n, false, s), vn = norm_sync(ctx, v, n, false, s);
                worst = std::max(worst, rn / (vn * std::max(std::abs(lam[i]), 1e-300)));
            }
            unpack_spinor(lat, E.vec(Rint, i), static_cast<char *>(Rout) + (size_t)i * nc * 16, SGN_PREC_F64, s);
            unpack_spinor(lat, E.vec(Lint, i), static_cast<char *>(Lout) + (size_t)i * nc * 16, SGN_PREC_F64, s);
            lambda[2 * i] = lam[i].real();
            lambda[2 * i + 1] = lam[i].imag();
        }
        SGN_HIP(hipStreamSynchronize(s));
        if (alpha) {  // smallest modulus among the accurate right Ritz values not selected (0 if none)
            double a = 0.0;
            for (size_t j = 0; j < rest_right.size(); ++j) a = (j == 0) ? rest_right[j] : std::min(a, rest_right[j]);
            *alpha = a;
        }
        record(worst);
        if (!converged) throw Failure{SGN_ERR_NOT_CONVERGED, "eigensolver: not converged within max_restarts"};
    });
}
