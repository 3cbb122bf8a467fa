// Multishift BiCG for the shifted systems of the Neuberger rational function,
// BiCG-LR(m) of the section "Two-sided Lanczos with rational functions".
//
// Systems: (A' - sigma_i) x_i = y,  A' = c^2 H_W(mu)^2,  y = c H_W (I - P) b.
// Seed: the shift of smallest modulus, M = A' - sigma_1, BiCG with shadow
// r~_0 = r_0.  The other shifts, M + tau_i (tau_i = sigma_1 - sigma_i), keep
// residuals collinear with the seed's, r^i_k = zeta^i_k r_k, with zeta from the
// three-term recurrence of the seed's residual polynomial.  Converged shifts
// are frozen (no more memory traffic).
//
// Precision schedule (mixed mode): while the seed residual is above theta32
// ||y|| everything is FP64; below it the vectors p_i, r, r~, p~ and the stencil
// drop to FP32 and the solutions accumulate in FP32 increments that are folded
// into FP64 x_i at every reliable update (true seed residual in FP64).  Below
// theta16 the stencil may also switch to FP16 links.  Rounding injected at a
// given iteration is proportional to the residual size at that point, so the
// shifted systems -- which get no reliable update -- keep residuals at the
// 1e-10 level without a separate refinement phase.
//
// Per iteration (all scalars on the device, host polls flags every few iterations):
//   tmp = A p;  q = c^2 A tmp - sigma_1 p   (+ partials of p~^H q)
//   tmp~ = A^H p~;  q~ = c^2 A^H tmp~ - sigma_1 p~
//   alpha = rho / p~^H q;  zeta^i_{k+1}, alpha_i          (1 block)
//   r -= alpha q;  r~ -= conj(alpha) q~   (+ partials of r~^H r, ||r||^2)
//   beta = rho'/rho;  beta_i = beta (zeta_{k+1}/zeta_k)^2; convergence flags (1 block)
//   x_i += alpha_i p_i;  p_i = zeta_{k+1} r + beta_i p_i;  p~ = r~ + conj(beta) p~
#include <algorithm>
#include <chrono>
#include <memory>
#include <vector>

#include "field_io.h"
#include "vec.h"

namespace sgn {

namespace {

constexpr int kS = SGN_MAX_POLES;

struct MsHead {
    z64 rho, alpha, beta, alpha_prev, beta_prev;
    double rnorm, rmax, ynorm, tol, delta, theta32, theta16;
    int done, reliable, want_phase, breakdown, iter, maxiter, nshift, seed, phase, pad;
};

struct MsState {
    MsHead h;
    z64 zeta[kS], zeta_prev[kS], zeta_next[kS], alpha_i[kS], beta_i[kS];    double tau[kS];
    double omega[kS];
    double res[kS];
    int act[kS], act_next[kS];
};

// Scalars of iteration k for shift i (zero when the shift was frozen): the
// stored-basis form rebuilds p_i and x_i from them.
struct MsHist {
    z64 alpha, beta, zeta;  // alpha_i^(k), beta_i^(k), zeta_i^(k+1)
};

__device__ __forceinline__ z64 cdiv(z64 a, z64 b)
{
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

__device__ __forceinline__ bool finite(z64 a) { return isfinite(a.r) && isfinite(a.i); }

__global__ void __launch_bounds__(256) ms_alpha_kernel(const z64 *partials, int nb, MsState *S)
{
    if (S->h.done) return;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        re += partials[i].r;
        im += partials[i].i;
    }
    __shared__ double lds[8];
    __shared__ z64 alpha_sh;
    __shared__ int bad_sh;
    double v[2] = {re, im};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        const z64 den = {v[0], v[1]};
        z64 a = cdiv(S->h.rho, den);
        bad_sh = 0;
        if (!(norm2(den) > 0.0) || !finite(a)) {
            S->h.breakdown = 1;
            S->h.done = 1;
            a = {0.0, 0.0};
            bad_sh = 1;
        }
        S->h.alpha = a;
        alpha_sh = a;
    }
    __syncthreads();
    if (bad_sh) return;
    const z64 al = alpha_sh, ap = S->h.alpha_prev, bp = S->h.beta_prev;
    for (int i = threadIdx.x; i < S->h.nshift; i += blockDim.x) {
        const int a = S->act_next[i];
        S->act[i] = a;
        if (!a) continue;
        const z64 z = S->zeta[i], zp = S->zeta_prev[i];
        const z64 one_tau = {1.0 + S->tau[i] * al.r, S->tau[i] * al.i};
        const z64 denom = ap * one_tau * zp + al * bp * (zp - z);
        const z64 zn = cdiv(z * zp * ap, denom);
        S->zeta_next[i] = zn;
        S->alpha_i[i] = cdiv(al * zn, z);
    }
}

__global__ void __launch_bounds__(256) ms_beta_kernel(const z64 *partials, int nb, MsState *S, MsHist *hist,
                                                      int hist_cap)
{
    if (S->h.done) return;
    const int k = S->h.iter;  // this iteration (read before thread 0 advances it)
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        a += partials[2 * i].r;
        b += partials[2 * i].i;
        c += partials[2 * i + 1].r;
    }
    __shared__ double lds[12];
    __shared__ z64 beta_sh;
    __shared__ double rn_sh;
    __shared__ int any_sh, bad_sh;
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        const z64 rho_new = {v[0], v[1]};
        z64 beta = cdiv(rho_new, S->h.rho);
        const double rn = sqrt(v[2]);
        bad_sh = 0;
        if (!(norm2(S->h.rho) > 0.0) || !finite(beta) || !isfinite(rn)) {
            S->h.breakdown = 1;
            S->h.done = 1;
            beta = {0.0, 0.0};
            bad_sh = 1;
        }
        S->h.beta = beta;
        S->h.rho = rho_new;
        S->h.rnorm = rn;
        S->h.rmax = fmax(S->h.rmax, rn);
        S->h.alpha_prev = S->h.alpha;
        S->h.beta_prev = beta;
        S->h.iter += 1;
        if (S->h.phase >= 1 && rn < S->h.delta * S->h.rmax) S->h.reliable = 1;
        if (S->h.phase == 0 && rn < S->h.theta32 * S->h.ynorm) S->h.want_phase = 1;
        if (S->h.phase == 1 && rn < S->h.theta16 * S->h.ynorm) S->h.want_phase = 2;
        beta_sh = beta;
        rn_sh = rn;
        any_sh = 0;
    }
    __syncthreads();
    if (bad_sh) return;
    const z64 beta = beta_sh;
    const double rn = rn_sh;
    const double lim = S->h.tol * S->h.ynorm;
    MsHist *hk = (hist && k < hist_cap) ? hist + (int64_t)k * S->h.nshift : nullptr;
    for (int i = threadIdx.x; i < S->h.nshift; i += blockDim.x) {
        if (!S->act[i]) {
            if (hk) hk[i] = MsHist{{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
            continue;
        }
        const z64 zn = S->zeta_next[i], z = S->zeta[i];
        const z64 q = cdiv(zn, z);
        S->beta_i[i] = beta * (q * q);
        if (hk) hk[i] = MsHist{S->alpha_i[i], S->beta_i[i], zn};
        S->zeta_prev[i] = z;
        S->zeta[i] = zn;
        const double ri = sqrt(norm2(zn)) * rn;
        S->res[i] = ri;
        const int an = ri > lim ? 1 : 0;
        S->act_next[i] = an;
        if (an) atomicOr(&any_sh, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!any_sh) {
            S->h.done = 1;
        } else {
            S->act_next[S->h.seed] = 1;  // the seed drives the recurrence
        }
        if (S->h.iter >= S->h.maxiter) S->h.done = 1;
    }
}

template <typename R> struct VecT;
template <> struct VecT<double> { using t = double2; };
template <> struct VecT<float> { using t = float2; };

template <typename T> __device__ __forceinline__ z64 ldz(const T *p, int64_t i)
{
    T v = p[i];
    return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stz(double2 *p, int64_t i, z64 v) { p[i] = make_double2(v.r, v.i); }
__device__ __forceinline__ void stz(float2 *p, int64_t i, z64 v) { p[i] = make_float2((float)v.r, (float)v.i); }

// r_out = r_in - alpha q (r_out may be r_in, or the next stored-basis slot),
// r~ -= conj(alpha) q~, with partials of r~^H r_out and ||r_out||^2
template <typename R>
__global__ void __launch_bounds__(256) ms_seed_update(const typename VecT<R>::t *r_in, typename VecT<R>::t *r_out,
                                                      typename VecT<R>::t *rt, const typename VecT<R>::t *q,
                                                      const typename VecT<R>::t *qt, int64_t n, const MsState *S,
                                                      z64 *partials)
{
    if (S->h.done) return;
    const z64 al = S->h.alpha, alc = conj(al);
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        z64 rv = ldz(r_in, e) - al * ldz(q, e);
        z64 tv = ldz(rt, e) - alc * ldz(qt, e);
        stz(r_out, e, rv);
        stz(rt, e, tv);
        if constexpr (sizeof(R) == 4) {  // reduce what is stored
            rv = ldz(r_out, e);
            tv = ldz(rt, e);
        }
        const z64 d = cmulc(tv, rv);
        a += d.r;
        b += d.i;
        c += norm2(rv);
    }
    __shared__ double lds[12];
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = {v[0], v[1]};
        partials[2 * blockIdx.x + 1] = {v[2], 0.0};
    }
}

// p_i = zeta_i r + beta_i p_i for the active shifts, p~ = r~ + conj(beta) p~, and the
// solution updates with the old p_i:
//   KEEP:  x_i += alpha_i p_i for every active shift (X holds s vectors)
//   else:  x_seed += alpha_seed p_seed and x_rest += sum_{i != seed} omega_i alpha_i p_i
//          (X holds 2 vectors) -- only the omega-weighted sum of the non-seed
//          solutions is ever needed, which halves the per-shift memory traffic.
template <typename R, typename XT, bool KEEP>
__global__ void __launch_bounds__(256) ms_shift_update(typename VecT<R>::t *P, XT *X, const typename VecT<R>::t *r,
                                                       const typename VecT<R>::t *rt, typename VecT<R>::t *pt,
                                                       int64_t n, const MsState *S, int expect,
                                                       unsigned long long *byte_counter)
{
    // apply only if this iteration's beta step ran (it may have just declared convergence;
    // later launches of a polling chunk after convergence must not repeat the update)
    if (S->h.breakdown || S->h.iter != expect) return;
    __shared__ z64 al_s[kS], be_s[kS], ze_s[kS];
    __shared__ int act_s[kS];
    __shared__ int ns, any_rest;
    const int nsh = S->h.nshift, seed = S->h.seed;
    if (threadIdx.x == 0) any_rest = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < nsh; i += blockDim.x) {
        const int a = S->act[i];
        act_s[i] = a;
        al_s[i] = (KEEP || i == seed) ? S->alpha_i[i] : S->omega[i] * S->alpha_i[i];
        be_s[i] = S->beta_i[i];
        ze_s[i] = S->zeta[i];
        if (a && i != seed) any_rest = 1;  // every writer stores the same value
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ns = nsh;
        if (byte_counter && blockIdx.x == 0) {  // algorithmic bytes of this launch (profiling)
            unsigned long long na = 0;
            for (int i = 0; i < nsh; ++i) na += act_s[i] ? 1 : 0;
            const unsigned long long eb = sizeof(typename VecT<R>::t), xb = sizeof(XT);
            const unsigned long long nxv = KEEP ? na : (1ull + (any_rest ? 1ull : 0ull));
            atomicAdd(byte_counter, (unsigned long long)n * (4ull * eb + na * 2ull * eb + nxv * 2ull * xb));
        }
    }
    __syncthreads();
    const z64 bc = conj(S->h.beta);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 rv = ldz(r, e);
        z64 rest = {0.0, 0.0};
        for (int i = 0; i < ns; ++i) {
            if (!act_s[i]) continue;
            typename VecT<R>::t *Pi = P + (int64_t)i * n;
            const z64 p = ldz(Pi, e);
            if (KEEP) {
                XT *Xi = X + (int64_t)i * n;
                stz(Xi, e, ldz(Xi, e) + al_s[i] * p);
            } else if (i == seed) {
                stz(X, e, ldz(X, e) + al_s[i] * p);
            } else {
                rest = rest + al_s[i] * p;
            }
            stz(Pi, e, ze_s[i] * rv + be_s[i] * p);
        }
        if (!KEEP && any_rest) stz(X + n, e, ldz(X + n, e) + rest);
        stz(pt, e, ldz(rt, e) + bc * ldz(pt, e));
    }
}

// Stored-basis form: only the seed keeps vectors,
//   x_seed += alpha p_seed;  p_seed = r + beta p_seed;  p~ = r~ + conj(beta) p~
// (zeta = 1 and alpha_i = alpha, beta_i = beta for the seed; the values are
// taken from the shift arrays all the same).
template <typename R, typename XT>
__global__ void __launch_bounds__(256) ms_seed_xp_update(typename VecT<R>::t *P, XT *X, const typename VecT<R>::t *r,
                                                         const typename VecT<R>::t *rt, typename VecT<R>::t *pt,
                                                         int64_t n, const MsState *S, int expect,
                                                         unsigned long long *byte_counter)
{
    if (S->h.breakdown || S->h.iter != expect) return;
    const int seed = S->h.seed;
    const z64 al = S->alpha_i[seed], be = S->beta_i[seed], ze = S->zeta[seed], bc = conj(S->h.beta);
    if (byte_counter && blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long eb = sizeof(typename VecT<R>::t), xb = sizeof(XT);
        atomicAdd(byte_counter, (unsigned long long)n * (6ull * eb + 2ull * xb));
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 p = ldz(P, e);
        stz(X, e, ldz(X, e) + al * p);
        stz(P, e, ze * ldz(r, e) + be * p);
        stz(pt, e, ldz(rt, e) + bc * ldz(pt, e));
    }
}

// out (+)= sum_j coef_j v_j over up to kLiftChunk stored vectors, FP64 or FP32 each.
// out and FP64 vectors use the [12][S] double2 layout; an FP32 vector is [6][S]
// float4, i.e. component c of site st is float2 entry 2 ((c/2) S + st) + c%2.
constexpr int kLiftChunk = 256;
struct LiftSlot {
    const void *p;
    int f32;
    int pad;
};

__global__ void __launch_bounds__(256) ms_lift_kernel(const LiftSlot *slots, const z64 *coef, int K, int Sst,
                                                      double2 *out, int accumulate)
{
    __shared__ LiftSlot sl[kLiftChunk];
    __shared__ z64 cf[kLiftChunk];
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        sl[j] = slots[j];
        cf[j] = coef[j];
    }
    __syncthreads();
    const int64_t n = (int64_t)12 * Sst;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int comp = (int)(e / Sst), st = (int)(e - (int64_t)comp * Sst);
        const int64_t e32 = 2 * ((int64_t)(comp >> 1) * Sst + st) + (comp & 1);
        z64 acc = {0.0, 0.0};
        if (accumulate) {
            const double2 o = out[e];
            acc = {o.x, o.y};
        }
        for (int j = 0; j < K; ++j) {
            const z64 c = cf[j];
            if (c.r == 0.0 && c.i == 0.0) continue;  // uniform
            const z64 v = sl[j].f32 ? ldz(static_cast<const float2 *>(sl[j].p), e32)
                                    : ldz(static_cast<const double2 *>(sl[j].p), e);
            acc = acc + c * v;
        }
        out[e] = make_double2(acc.r, acc.i);
    }
}

// x_hi_i += x_lo_i ; x_lo_i = 0   (FP32 layout -> FP64 layout, pair mapping)
__global__ void ms_flush_kernel(double2 *Xhi, float4 *Xlo, int s, int V /* component stride */)
{
    const int64_t np = (int64_t)6 * V;
    const int64_t n = (int64_t)12 * V;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(p / V), st = (int)(p - (int64_t)c2 * V);
        const int64_t e0 = (int64_t)(2 * c2) * V + st, e1 = e0 + V;
        for (int i = 0; i < s; ++i) {
            float4 l = Xlo[(int64_t)i * np + p];
            double2 *h = Xhi + (int64_t)i * n;
            double2 a = h[e0], b = h[e1];
            h[e0] = make_double2(a.x + l.x, a.y + l.y);
            h[e1] = make_double2(b.x + l.z, b.y + l.w);
            Xlo[(int64_t)i * np + p] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

// r32 = f32(y + t) (pair mapping) with partials of rt32^H r32 and ||r32||^2
__global__ void __launch_bounds__(256) ms_reliable_kernel(const double2 *y, const double2 *t, float4 *r32,
                                                          const float4 *rt32, int V /* component stride */,
                                                          z64 *partials)
{
    const int64_t np = (int64_t)6 * V;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(p / V), st = (int)(p - (int64_t)c2 * V);
        const int64_t e0 = (int64_t)(2 * c2) * V + st, e1 = e0 + V;
        const double2 y0 = y[e0], y1 = y[e1], t0 = t[e0], t1 = t[e1];
        const float4 rv = make_float4((float)(y0.x + t0.x), (float)(y0.y + t0.y), (float)(y1.x + t1.x),
                                      (float)(y1.y + t1.y));
        r32[p] = rv;
        const float4 tv = rt32[p];
        a += (double)tv.x * rv.x + (double)tv.y * rv.y + (double)tv.z * rv.z + (double)tv.w * rv.w;
        b += (double)tv.x * rv.y - (double)tv.y * rv.x + (double)tv.z * rv.w - (double)tv.w * rv.z;
        c += (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z + (double)rv.w * rv.w;
    }
    __shared__ double lds[12];
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = {v[0], v[1]};
        partials[2 * blockIdx.x + 1] = {v[2], 0.0};
    }
}

__global__ void __launch_bounds__(256) ms_reliable_coef(const z64 *partials, int nb, MsState *S)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        a += partials[2 * i].r;
        b += partials[2 * i].i;
        c += partials[2 * i + 1].r;
    }
    __shared__ double lds[12];
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        S->h.rho = {v[0], v[1]};
        const double rn = sqrt(v[2]);
        S->h.rnorm = rn;
        S->h.rmax = rn;
        S->h.reliable = 0;
        const int seed = S->h.seed;
        S->res[seed] = rn;
        if (rn > S->h.tol * S->h.ynorm && S->h.iter < S->h.maxiter) {
            S->act_next[seed] = 1;
            S->h.done = 0;
        }
    }
}

// x = sum_i w_i X_i (FP64)
__global__ void ms_combine_kernel(const double2 *X, const double *w, int s, int64_t n, double2 *x)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < s; ++i) {
            const double2 v = X[(int64_t)i * n + e];
            re += w[i] * v.x;
            im += w[i] * v.y;
        }
        x[e] = make_double2(re, im);
    }
}

template <typename T>
__global__ void fill_kernel(T *p, T v, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

__global__ void copy_rep_kernel(const double2 *src, double2 *dst, int s, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = src[e];
        for (int i = 0; i < s; ++i) dst[(int64_t)i * n + e] = v;
    }
}

struct DevMem {
    void *p = nullptr;
    explicit DevMem(size_t bytes)
    {
        if (bytes && hipMalloc(&p, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "multishift workspace"};
    }
    ~DevMem()
    {
        if (p) (void)hipFree(p);
    }
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct Span {
    void *p;
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Coefficients of the stored residuals r_0..r_k for shift i from the scalar
// history (iterations 0..k-1):
//   p_i^(k) = sum_{j<=k} a_j r_j,  a_j = zeta^(j) prod_{l=j}^{k-1} beta^(l)
//   x_i^(k) = sum_{j<k}  c_j r_j,  c_j = zeta^(j) g^(j),  g^(j) = alpha^(j) + beta^(j) g^(j+1),  g^(k) = 0
// where zeta^(0) = 1 and zeta^(j) is the zeta recorded at iteration j-1.
void basis_coefficients(const std::vector<MsHist> &H, int ns, int k, int i, std::vector<z64> *c,
                        std::vector<z64> *a)
{
    auto zeta = [&](int j) -> z64 { return j == 0 ? z64{1.0, 0.0} : H[(size_t)(j - 1) * ns + i].zeta; };
    if (c) {
        c->assign(k, z64{0.0, 0.0});
        z64 g = {0.0, 0.0};
        for (int j = k - 1; j >= 0; --j) {
            const MsHist &h = H[(size_t)j * ns + i];
            g = h.alpha + h.beta * g;
            (*c)[j] = zeta(j) * g;
        }
    }
    if (a) {
        a->assign(k + 1, z64{0.0, 0.0});
        (*a)[k] = zeta(k);
        z64 prod = {1.0, 0.0};
        for (int j = k - 1; j >= 0; --j) {
            prod = prod * H[(size_t)j * ns + i].beta;
            (*a)[j] = zeta(j) * prod;
        }
    }
}

// One problem of multishift_solve.
sgn_status solve_one(const sgn_problem &pb, const sgn_rational &rf, const sgn_ms_opts &o, sgn_stats *st,
                     hipStream_t s)
{
    const auto t_start = std::chrono::steady_clock::now();
    Lattice &lat = *as_lattice(pb.lat);
    Context &ctx = *lat.ctx;
    SGN_HIP(hipSetDevice(ctx.device));
    // internal vectors have n = 12 S entries (padded component stride), canonical ones nc = 12 V
    const int64_t V = lat.V, Sst = lat.S, n = 12 * Sst, nc = 12 * V;
    const size_t b64 = (size_t)n * 16, b32 = (size_t)n * 8, c64 = (size_t)nc * 16;
    const int ns = rf.s;
    const bool mixed = o.prec != SGN_PREC_F64;
    const double c2 = rf.c * rf.c;
    int seed = 0;
    for (int i = 1; i < ns; ++i)
        if (std::abs(rf.sigma[i]) < std::abs(rf.sigma[seed])) seed = i;
    const double s1 = rf.sigma[seed];
    const int maxiter = o.maxiter > 0 ? o.maxiter : 10000;

    // Stored-basis form unless per-shift solutions are wanted: slots 1..slot_cap
    // may hold residuals r_j (slot 0 is y itself).
    const bool want_shifts = pb.x_shift != nullptr || o.verify;
    int slot_cap = 0;
    if (!want_shifts && o.basis_slots >= 0) {
        if (o.basis_slots > 0) {
            slot_cap = o.basis_slots;
        } else {
            size_t fr = 0, tot = 0;
            SGN_HIP(hipMemGetInfo(&fr, &tot));
            slot_cap = (int)std::min<double>(1e9, 0.5 * (double)(fr + ctx.basis_bytes()) / (double)b64);
        }
        slot_cap = std::min(slot_cap, maxiter);
    }
    bool explicit_mode = slot_cap < 1;
    const int np0 = explicit_mode ? ns : 1;  // p and x vectors held in the arena
    const size_t hist_bytes = explicit_mode ? 0 : (size_t)slot_cap * ns * sizeof(MsHist);

    // workspace carved from the context's arena (kept between calls)
    const size_t a64 = (8 + 2 * (size_t)np0) * b64 + c64, a32 = mixed ? (7 + 2 * (size_t)np0) * b32 : 0;
    char *arena = static_cast<char *>(ctx.ensure_arena(a64 + a32 + hist_bytes + sizeof(MsState)));
    auto carve = [&](size_t bytes) {
        Span sp{arena};
        arena += bytes;
        return sp;
    };
    Span y = carve(b64), r = carve(b64), rt = carve(b64), pt = carve(b64), q = carve(b64), qt = carve(b64),
         tmp = carve(b64), tmpt = carve(b64);
    Span X = carve((size_t)np0 * b64), P = carve((size_t)np0 * b64);
    Span r32 = carve(mixed ? b32 : 0), rt32 = carve(mixed ? b32 : 0), pt32 = carve(mixed ? b32 : 0),
         q32 = carve(mixed ? b32 : 0), qt32 = carve(mixed ? b32 : 0), tmp32 = carve(mixed ? b32 : 0),
         tmpt32 = carve(mixed ? b32 : 0);
    Span P32 = carve(mixed ? (size_t)np0 * b32 : 0), Xlo = carve(mixed ? (size_t)np0 * b32 : 0);
    MsHist *hist = carve(hist_bytes).as<MsHist>();
    MsState *S = carve(sizeof(MsState)).as<MsState>();
    Span rcan = carve(c64);
    std::unique_ptr<DevMem> xp64, xp32;  // per-shift vectors after a change to explicit form

    // x <- x_P, r = (I - P) b (canonical)
    deflation_prologue(ctx, pb.defl, nc, pb.b, pb.x, rcan.p, nullptr, s);

    OpSpec opA, opAh;
    opA.mu = pb.mu;
    opAh.mu = -pb.mu;
    // y = c A r
    pack_spinor(lat, rcan.p, tmp.p, SGN_PREC_F64, s);
    {
        Epilogue ep;
        ep.a = rf.c;
        dslash_launch(lat, SGN_PREC_F64, opA, tmp.p, y.p, ep, s);
    }
    const double ynorm = norm_sync(ctx, y.p, n, false, s);
    SGN_REQUIRE(std::isfinite(ynorm), "multishift_solve: b contains NaN or Inf");
    if (st) {
        *st = sgn_stats{};
        st->nshift = ns;
    }
    if (ynorm == 0.0) return SGN_OK;  // x = x_P

    const int nvb = vec_blocks(n);
    const int nst = dslash_blocks(lat);
    const int nvbp = vec_blocks(6 * Sst);
    z64 *part = static_cast<z64 *>(ctx.ensure_partials(sizeof(z64) * std::max({nst, 2 * nvb, 2 * nvbp})));

    // initial state
    MsState h0{};
    h0.h.rho = {ynorm * ynorm, 0.0};
    h0.h.alpha_prev = {1.0, 0.0};
    h0.h.beta_prev = {0.0, 0.0};
    h0.h.rnorm = h0.h.rmax = h0.h.ynorm = ynorm;
    h0.h.tol = o.tol;
    h0.h.delta = o.delta > 0 ? o.delta : 0.1;
    h0.h.theta32 = mixed ? (o.theta32 > 0 ? o.theta32 : 1e-3) : 0.0;
    h0.h.theta16 = (o.prec == SGN_PREC_F32_H16) ? (o.theta16 > 0 ? o.theta16 : 1e-6) : 0.0;
    h0.h.maxiter = maxiter;
    h0.h.nshift = ns;
    h0.h.seed = seed;
    for (int i = 0; i < ns; ++i) {
        h0.zeta[i] = h0.zeta_prev[i] = {1.0, 0.0};
        h0.tau[i] = s1 - rf.sigma[i];
        h0.omega[i] = rf.omega[i];
        h0.act_next[i] = 1;
        h0.res[i] = ynorm;
    }
    SGN_HIP(hipMemcpyAsync(S, &h0, sizeof(MsState), hipMemcpyHostToDevice, s));
    SGN_HIP(hipMemcpyAsync(r.p, y.p, b64, hipMemcpyDeviceToDevice, s));
    SGN_HIP(hipMemcpyAsync(rt.p, y.p, b64, hipMemcpyDeviceToDevice, s));
    SGN_HIP(hipMemcpyAsync(pt.p, y.p, b64, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(copy_rep_kernel, dim3(nvb), dim3(256), 0, s, y.as<double2>(), P.as<double2>(), np0, n);
    hipLaunchKernelGGL(fill_kernel<double2>, dim3(nvb), dim3(256), 0, s, X.as<double2>(), make_double2(0, 0),
                       (int64_t)np0 * n);
    SGN_HIP(hipGetLastError());

    int phase = 0;
    int poll = o.poll > 0 ? o.poll : (int)std::min<int64_t>(16, std::max<int64_t>(1, (200000 + V - 1) / V));
    int reliable_updates = 0;
    const double sigma_seed = s1;

    // stored basis: slot j holds the residual r_j written by iteration j-1
    std::vector<char> slot_f32(1, 0);
    auto slot_ptr = [&](int j) -> void * { return j == 0 ? y.p : ctx.basis[(size_t)j - 1]; };
    void *cur = y.p;  // residual the next seed update starts from (basis form)

    int launched = 0;  // iteration number of the next launch minus one (synced with the device at polls)
    auto iterate = [&](int count) {
        for (int it = 0; it < count; ++it) {
            ++launched;
            const bool lo = phase >= 1;
            const sgn_prec sp = phase == 0 ? SGN_PREC_F64 : (phase == 1 ? SGN_PREC_F32 : SGN_PREC_F32_H16);
            const size_t pso = explicit_mode ? (size_t)seed : 0;  // seed's index in P / X
            void *pseed = lo ? (void *)(P32.as<char>() + pso * b32) : (void *)(P.as<char>() + pso * b64);
            void *vrt = lo ? rt32.p : rt.p, *vpt = lo ? pt32.p : pt.p;
            void *vq = lo ? q32.p : q.p, *vqt = lo ? qt32.p : qt.p, *vtmp = lo ? tmp32.p : tmp.p,
                 *vtmpt = lo ? tmpt32.p : tmpt.p;
            void *rin, *rout;
            if (explicit_mode) {
                rin = rout = lo ? r32.p : r.p;
            } else {
                rin = cur;
                rout = slot_ptr(launched);
                if ((int)slot_f32.size() <= launched) slot_f32.resize(launched + 1, 0);
                slot_f32[launched] = lo ? 1 : 0;
                cur = rout;
            }
            dslash_launch(lat, sp, opA, pseed, vtmp, Epilogue{}, s);
            Epilogue e1;
            e1.a = c2;
            e1.z = pseed;
            e1.b = {-sigma_seed, 0.0};
            e1.w = vpt;
            e1.partials = part;
            const int nb1 = dslash_launch(lat, sp, opA, vtmp, vq, e1, s);
            dslash_launch(lat, sp, opAh, vpt, vtmpt, Epilogue{}, s);
            Epilogue e2;
            e2.a = c2;
            e2.z = vpt;
            e2.b = {-sigma_seed, 0.0};
            dslash_launch(lat, sp, opAh, vtmpt, vqt, e2, s);
            hipLaunchKernelGGL(ms_alpha_kernel, dim3(1), dim3(256), 0, s, part, nb1, S);
            unsigned long long *bc = ctx.prof ? ctx.byte_counter : nullptr;
            const double eb = lo ? 8.0 : 16.0;
            int pr = ctx.prof_start(s);
            if (lo)
                hipLaunchKernelGGL(ms_seed_update<float>, dim3(nvb), dim3(256), 0, s, (const float2 *)rin,
                                   (float2 *)rout, (float2 *)vrt, (const float2 *)vq, (const float2 *)vqt, n, S, part);
            else
                hipLaunchKernelGGL(ms_seed_update<double>, dim3(nvb), dim3(256), 0, s, (const double2 *)rin,
                                   (double2 *)rout, (double2 *)vrt, (const double2 *)vq, (const double2 *)vqt, n, S,
                                   part);
            ctx.prof_stop(pr, s, SGN_K_SEED_UPDATE, 6.0 * eb * n, 40.0 * n);
            hipLaunchKernelGGL(ms_beta_kernel, dim3(1), dim3(256), 0, s, part, nvb, S,
                               explicit_mode ? nullptr : hist, explicit_mode ? 0 : slot_cap);
            pr = ctx.prof_start(s);
            if (!explicit_mode) {
                if (lo)
                    hipLaunchKernelGGL((ms_seed_xp_update<float, float2>), dim3(nvb), dim3(256), 0, s,
                                       P32.as<float2>(), Xlo.as<float2>(), (const float2 *)rout, (const float2 *)vrt,
                                       (float2 *)vpt, n, S, launched, bc);
                else
                    hipLaunchKernelGGL((ms_seed_xp_update<double, double2>), dim3(nvb), dim3(256), 0, s,
                                       P.as<double2>(), X.as<double2>(), (const double2 *)rout, (const double2 *)vrt,
                                       (double2 *)vpt, n, S, launched, bc);
            } else if (lo) {
                hipLaunchKernelGGL((ms_shift_update<float, float2, true>), dim3(nvb), dim3(256), 0, s,
                                   P32.as<float2>(), Xlo.as<float2>(), (const float2 *)rout, (const float2 *)vrt,
                                   (float2 *)vpt, n, S, launched, bc);
            } else {
                hipLaunchKernelGGL((ms_shift_update<double, double2, true>), dim3(nvb), dim3(256), 0, s,
                                   P.as<double2>(), X.as<double2>(), (const double2 *)rout, (const double2 *)vrt,
                                   (double2 *)vpt, n, S, launched, bc);
            }
            ctx.prof_stop(pr, s, SGN_K_SHIFT_UPDATE, 0.0, 0.0, true);
        }
        SGN_HIP(hipGetLastError());
    };

    auto nxv = [&]() { return explicit_mode ? ns : 1; };
    auto flush = [&]() {
        hipLaunchKernelGGL(ms_flush_kernel, dim3(nvbp), dim3(256), 0, s, X.as<double2>(), Xlo.as<float4>(), nxv(),
                           (int)Sst);
    };

    auto reliable_update = [&]() {
        flush();
        double2 *xs = X.as<double2>() + (explicit_mode ? (size_t)seed * n : 0);
        dslash_launch(lat, SGN_PREC_F64, opA, xs, tmp.p, Epilogue{}, s);
        Epilogue ep;
        ep.a = -c2;
        ep.z = xs;
        ep.b = {sigma_seed, 0.0};
        dslash_launch(lat, SGN_PREC_F64, opA, tmp.p, q.p, ep, s);  // q = -c^2 A A x + sigma x
        hipLaunchKernelGGL(ms_reliable_kernel, dim3(nvbp), dim3(256), 0, s, y.as<double2>(), q.as<double2>(),
                           r32.as<float4>(), rt32.as<float4>(), (int)Sst, part);
        hipLaunchKernelGGL(ms_reliable_coef, dim3(1), dim3(256), 0, s, part, nvbp, S);
        SGN_HIP(hipGetLastError());
        if (!explicit_mode) cur = r32.p;
        ++reliable_updates;
    };

    auto switch_to_f32 = [&]() {
        convert_64_to_32(explicit_mode ? r.p : cur, r32.p, Sst, s);
        if (!explicit_mode) cur = r32.p;
        convert_64_to_32(rt.p, rt32.p, Sst, s);
        convert_64_to_32(pt.p, pt32.p, Sst, s);
        for (int i = 0; i < nxv(); ++i)
            convert_64_to_32(P.as<char>() + (size_t)i * b64, P32.as<char>() + (size_t)i * b32, Sst, s);
        hipLaunchKernelGGL(fill_kernel<float2>, dim3(nvb), dim3(256), 0, s, Xlo.as<float2>(), make_float2(0, 0),
                           (int64_t)nxv() * n);
        SGN_HIP(hipGetLastError());
    };

    // out (+)= sum_j coef[j] slot_j over slots 0..K-1
    auto lift = [&](const std::vector<z64> &coef, void *out, bool accumulate) {
        const int K = (int)coef.size();
        std::vector<LiftSlot> hs(K);
        double bytes = accumulate ? 2.0 * b64 : (double)b64;
        for (int j = 0; j < K; ++j) {
            hs[j] = LiftSlot{slot_ptr(j), slot_f32[j], 0};
            bytes += (coef[j].r != 0.0 || coef[j].i != 0.0) ? (slot_f32[j] ? (double)b32 : (double)b64) : 0.0;
        }
        DevMem dsl(sizeof(LiftSlot) * std::max(K, 1)), dcf(sizeof(z64) * std::max(K, 1));
        SGN_HIP(hipMemcpy(dsl.p, hs.data(), sizeof(LiftSlot) * K, hipMemcpyHostToDevice));
        SGN_HIP(hipMemcpy(dcf.p, coef.data(), sizeof(z64) * K, hipMemcpyHostToDevice));
        const int pr = ctx.prof_start(s);
        bool acc = accumulate;
        for (int j0 = 0; j0 < K || (j0 == 0 && !acc); j0 += kLiftChunk) {
            const int kk = std::min(kLiftChunk, K - j0);
            hipLaunchKernelGGL(ms_lift_kernel, dim3(nvb), dim3(256), 0, s, dsl.as<LiftSlot>() + j0,
                               dcf.as<z64>() + j0, kk, (int)Sst, static_cast<double2 *>(out), acc ? 1 : 0);
            acc = true;
            if (K == 0) break;
        }
        SGN_HIP(hipGetLastError());
        ctx.prof_stop(pr, s, SGN_K_LIFT, bytes, 8.0 * n * K);
        SGN_HIP(hipStreamSynchronize(s));  // dsl, dcf go out of scope
    };
    auto history = [&](int k) {
        std::vector<MsHist> H((size_t)k * ns);
        if (k > 0) SGN_HIP(hipMemcpy(H.data(), hist, sizeof(MsHist) * H.size(), hipMemcpyDeviceToHost));
        return H;
    };

    // Turn the stored basis into explicit p_i, x_i at iteration k = launched
    // (all launched iterations have run) and continue with per-shift vectors.
    auto to_explicit = [&]() {
        const int k = launched;
        const std::vector<MsHist> H = history(k);
        xp64 = std::make_unique<DevMem>(2 * (size_t)ns * b64);
        if (mixed) xp32 = std::make_unique<DevMem>(2 * (size_t)ns * b32);
        Span Xn{xp64->p}, Pn{xp64->as<char>() + (size_t)ns * b64};
        Span Xlon{mixed ? xp32->p : nullptr}, P32n{mixed ? xp32->as<char>() + (size_t)ns * b32 : nullptr};
        if (phase >= 1) flush();
        std::vector<z64> cj, aj;
        for (int i = 0; i < ns; ++i) {
            char *xi = Xn.as<char>() + (size_t)i * b64, *pi = Pn.as<char>() + (size_t)i * b64;
            if (i == seed) {
                SGN_HIP(hipMemcpyAsync(xi, X.p, b64, hipMemcpyDeviceToDevice, s));
                if (phase >= 1)
                    SGN_HIP(hipMemcpyAsync(P32n.as<char>() + (size_t)i * b32, P32.p, b32, hipMemcpyDeviceToDevice, s));
                else
                    SGN_HIP(hipMemcpyAsync(pi, P.p, b64, hipMemcpyDeviceToDevice, s));
                continue;
            }
            basis_coefficients(H, ns, k, i, &cj, &aj);
            lift(cj, xi, false);
            lift(aj, pi, false);
            if (phase >= 1) convert_64_to_32(pi, P32n.as<char>() + (size_t)i * b32, Sst, s);
        }
        if (mixed)
            hipLaunchKernelGGL(fill_kernel<float2>, dim3(nvb), dim3(256), 0, s, Xlon.as<float2>(), make_float2(0, 0),
                               (int64_t)ns * n);
        // the explicit form keeps the current residual in r (FP64) or r32
        if (phase >= 1) {
            if (cur != r32.p) SGN_HIP(hipMemcpyAsync(r32.p, cur, b32, hipMemcpyDeviceToDevice, s));
        } else {
            SGN_HIP(hipMemcpyAsync(r.p, cur, b64, hipMemcpyDeviceToDevice, s));
        }
        SGN_HIP(hipStreamSynchronize(s));
        X = Xn;
        P = Pn;
        Xlo = Xlon;
        P32 = P32n;
        explicit_mode = true;
    };

    MsHead hh{};
    auto read_head = [&]() {
        SGN_HIP(hipMemcpyAsync(&hh, &S->h, sizeof(MsHead), hipMemcpyDeviceToHost, s));
        SGN_HIP(hipStreamSynchronize(s));
        launched = hh.iter;
    };
    auto put = [&](void *dst, const void *src, size_t bytes) {
        SGN_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        SGN_HIP(hipStreamSynchronize(s));
    };
    auto set_phase = [&](int ph) {
        phase = ph;
        const int zero = 0;
        put(&S->h.phase, &ph, sizeof(int));
        put(&S->h.want_phase, &zero, sizeof(int));
    };

    const auto t_kry = std::chrono::steady_clock::now();
    sgn_status result = SGN_OK;
    for (;;) {
        if (!explicit_mode) {
            // slots for the next chunk; past the budget the basis becomes explicit vectors
            const int upto = launched + poll;
            if (upto > slot_cap || !ctx.ensure_basis(upto - 1, b64)) to_explicit();
        }
        const int iter_before = launched;
        iterate(poll);
        read_head();
        if (!explicit_mode && hh.iter > iter_before) cur = slot_ptr(hh.iter);
        if (hh.breakdown) throw Failure{SGN_ERR_BREAKDOWN, "multishift BiCG breakdown at iteration " + std::to_string(hh.iter)};
        if (hh.done) {
            if (phase >= 1) {
                reliable_update();
                read_head();
                if (!hh.done) continue;
            }
            if (hh.iter >= maxiter && hh.rnorm > o.tol * ynorm) result = SGN_ERR_NOT_CONVERGED;
            break;
        }
        if (mixed && hh.want_phase > phase) {
            if (phase == 0) {
                switch_to_f32();
                set_phase(1);
                const double rm = hh.rnorm;
                put(&S->h.rmax, &rm, sizeof(double));
            } else if (phase == 1 && o.prec == SGN_PREC_F32_H16) {
                set_phase(2);
            }
            continue;
        }
        if (phase >= 1 && hh.reliable) reliable_update();
    }
    if (phase >= 1) flush();
    const double kry_ms = ms_since(t_kry);

    // x += sum_i omega_i x_i
    {
        if (explicit_mode) {
            DevMem w(sizeof(double) * ns);
            SGN_HIP(hipMemcpy(w.p, rf.omega, sizeof(double) * ns, hipMemcpyHostToDevice));
            hipLaunchKernelGGL(ms_combine_kernel, dim3(nvb), dim3(256), 0, s, X.as<double2>(), w.as<double>(), ns, n,
                               tmp.as<double2>());
            SGN_HIP(hipGetLastError());
            SGN_HIP(hipStreamSynchronize(s));
        } else {
            // omega_seed x_seed + sum_j d_j r_j,  d_j = sum_{i != seed} omega_i c_ij
            const int K = launched;
            const std::vector<MsHist> H = history(K);
            std::vector<z64> d(K, z64{0.0, 0.0}), cj;
            for (int i = 0; i < ns; ++i) {
                if (i == seed) continue;
                basis_coefficients(H, ns, K, i, &cj, nullptr);
                for (int j = 0; j < K; ++j) d[j] = d[j] + rf.omega[i] * cj[j];
            }
            scale64({rf.omega[seed], 0.0}, X.p, tmp.p, n, s);
            lift(d, tmp.p, true);
        }
        unpack_spinor(lat, tmp.p, rcan.p, SGN_PREC_F64, s);
        axpby64({1.0, 0.0}, rcan.p, {1.0, 0.0}, pb.x, nc, s);
        if (pb.x_shift)
            for (int i = 0; i < ns; ++i)
                if (pb.x_shift[i]) unpack_spinor(lat, X.as<char>() + (size_t)i * b64, pb.x_shift[i], SGN_PREC_F64, s);
        SGN_HIP(hipStreamSynchronize(s));
    }
    if (st) {
        MsState hs;
        SGN_HIP(hipMemcpy(&hs, S, sizeof(MsState), hipMemcpyDeviceToHost));
        st->iterations = hs.h.iter;
        st->matvecs = 4 * hs.h.iter + 1 + 2 * reliable_updates;
        st->reliable_updates = reliable_updates;
        double mx = 0.0;
        for (int i = 0; i < ns; ++i) {
            st->shift_residual[i] = hs.res[i] / ynorm;
            mx = std::max(mx, st->shift_residual[i]);
        }
        if (o.verify) {  // FP64 true residuals of every shifted system
            mx = 0.0;
            for (int i = 0; i < ns; ++i) {
                double2 *xi = X.as<double2>() + (size_t)i * n;
                dslash_launch(lat, SGN_PREC_F64, opA, xi, tmp.p, Epilogue{}, s);
                Epilogue ep;
                ep.a = -c2;
                ep.z = xi;
                ep.b = {rf.sigma[i], 0.0};
                dslash_launch(lat, SGN_PREC_F64, opA, tmp.p, q.p, ep, s);
                axpby64({1.0, 0.0}, y.p, {1.0, 0.0}, q.p, n, s);
                st->shift_residual[i] = norm_sync(ctx, q.p, n, false, s) / ynorm;
                mx = std::max(mx, st->shift_residual[i]);
            }
            st->matvecs += 2 * ns;
        }
        st->residual = mx;
        st->krylov_ms = kry_ms;
        st->total_ms = ms_since(t_start);
    }
    return result;
}

}  // namespace

}  // namespace sgn

using namespace sgn;

extern "C" sgn_status multishift_solve(const sgn_problem *pb, int nprob, const sgn_rational *rf,
                                       const sgn_ms_opts *o, sgn_stats *stats, void *stream)
{
    sgn_status worst = SGN_OK;
    sgn_status st = guard([&] {
        SGN_REQUIRE(pb && rf && o && nprob >= 0, "multishift_solve: null argument");
        SGN_REQUIRE(rf->s >= 1 && rf->s <= SGN_MAX_POLES, "multishift_solve: bad number of poles");
        SGN_REQUIRE(rf->c > 0 && std::isfinite(rf->c), "multishift_solve: bad scale c");
        for (int i = 0; i < rf->s; ++i)
            SGN_REQUIRE(rf->sigma[i] < 0 && std::isfinite(rf->omega[i]), "multishift_solve: shifts must be negative");
        SGN_REQUIRE(o->tol > 0 && o->tol < 1, "multishift_solve: tol must be in (0, 1)");
        for (int p = 0; p < nprob; ++p) {
            SGN_REQUIRE(pb[p].lat && pb[p].b && pb[p].x, "multishift_solve: null problem field");
            SGN_REQUIRE(std::isfinite(pb[p].mu), "multishift_solve: mu not finite");
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        for (int p = 0; p < nprob; ++p) {
            const sgn_status r = solve_one(pb[p], *rf, *o, stats ? &stats[p] : nullptr, s);
            if (r != SGN_OK && worst == SGN_OK) worst = r;
        }
    });
    return st != SGN_OK ? st : worst;
}
