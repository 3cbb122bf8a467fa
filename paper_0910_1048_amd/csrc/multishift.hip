// Multishift BiCG for the shifted systems of the Neuberger rational function,
// BiCG-LR(m) of the section "Two-sided Lanczos with rational functions".
//
// Systems: (A' - sigma_i) x_i = y,  A' = c^2 H_W(mu)^2,  y = c H_W (I - P) b.
// Seed: the shift of smallest modulus, M = A' - sigma_1, BiCG with shadow
// r~_0 = r_0.  The other shifts, M + tau_i (tau_i = sigma_1 - sigma_i), keep
// residuals collinear with the seed's, r^i_k = zeta^i_k r_k, with zeta from the
// three-term recurrence of the seed's residual polynomial.  Converged shifts
// are frozen.
//
// Two forms of the same iteration:
//  * stored basis (default when per-shift solutions are not requested): every
//    seed residual r_k is kept in its own slot; p_i and x_i of the non-seed
//    shifts are linear combinations of the r_k whose coefficients follow from
//    the recorded scalars, so only the seed keeps p and x, and the
//    omega-weighted sum of the other solutions is one lift at the end;
//  * per-shift vectors: p_i and x_i of every shift are updated each iteration.
//
// Precision schedule (mixed mode): while the seed residual is above theta32
// ||y|| everything is FP64; below it the vectors and the stencil drop to FP32
// and the solutions accumulate in FP32 increments that are folded into FP64 at
// every reliable update (true seed residual in FP64).  Below theta16 the
// stencil may also switch to FP16 links.  Rounding injected at a given
// iteration is proportional to the residual size at that point, so the
// shifted systems -- which get no reliable update -- keep residuals at the
// 1e-10 level without a separate refinement phase.
//
// Batching: all problems of one call iterate in lockstep.  Each step of an
// iteration is one launch over every problem in the same precision phase
// (blockIdx.y selects the problem, whose pointers sit in a device-side
// descriptor); the host polls all of them every few iterations.
//
// Per iteration (all scalars on the device):
//   tmp = A p;  q = c^2 A tmp - sigma_1 p   (+ partials of p~^H q)
//   tmp~ = A^H p~;  q~ = c^2 A^H tmp~ - sigma_1 p~
//   alpha = rho / p~^H q;  zeta^i_{k+1}, alpha_i          (1 block per problem)
//   r_{k+1} = r_k - alpha q;  r~ -= conj(alpha) q~   (+ partials of r~^H r, ||r||^2)
//   beta = rho'/rho;  beta_i = beta (zeta_{k+1}/zeta_k)^2; convergence flags
//   x_i += alpha_i p_i;  p_i = zeta_{k+1} r + beta_i p_i;  p~ = r~ + conj(beta) p~
#include <algorithm>
#include <chrono>
#include <complex>
#include <memory>
#include <vector>

#include "field_io.h"
#include "vec.h"

namespace sgn {

namespace {

constexpr int kS = SGN_MAX_POLES;
constexpr int kVecGrid = 1024;  // blocks of the batched vector kernels (grid-stride over each problem)

struct MsHead {
    z64 rho, alpha, beta, alpha_prev, beta_prev;
    double rnorm, rmax, ynorm, tol, delta, theta32, theta16;
    int done, reliable, want_phase, breakdown, iter, maxiter, nshift, seed, phase;
    int go;  // set by the beta step of an iteration: that iteration's solution/direction update may run
};

struct MsState;
__global__ void __launch_bounds__(64) ms_gather_heads(MsState *const *S, MsHead *out);

struct MsState {
    MsHead h;
    z64 zeta[kS], zeta_prev[kS], zeta_next[kS], alpha_i[kS], beta_i[kS];
    double tau[kS];
    double omega[kS];
    double res[kS];
    int act[kS], act_next[kS];
};

// the heads of a batch's problems into one array (one copy to the host per chunk)
static_assert(sizeof(MsHead) % 8 == 0, "MsHead is copied in 8-byte words");
__global__ void __launch_bounds__(64) ms_gather_heads(MsState *const *S, MsHead *out)
{
    const uint64_t *src = reinterpret_cast<const uint64_t *>(&S[blockIdx.x]->h);
    uint64_t *dst = reinterpret_cast<uint64_t *>(out + blockIdx.x);
    for (int i = threadIdx.x; i < (int)(sizeof(MsHead) / 8); i += blockDim.x) dst[i] = src[i];
}

// Scalars of iteration k for shift i (zero when the shift was frozen): the
// stored-basis form rebuilds p_i and x_i from them.
struct MsHist {
    z64 alpha, beta, zeta;  // alpha_i^(k), beta_i^(k), zeta_i^(k+1)
};

// Device-side descriptor of one problem for the batched iteration kernels.
// The vector pointers are those of the problem's current precision.
struct MsVec {
    MsState *S;
    void *r;             // per-shift form: the residual (updated in place); stored-basis form: the
                         // residual that replaces slot temp_iter as input (after a reliable update)
    void *const *slots;  // stored-basis form: slot table, slot 0 = y; nullptr in per-shift form
    int temp_iter;       // stored-basis form: iteration whose seed update starts from r
    int nst_part;        // partials written by the dotting stencil
    void *rt, *q, *qt, *pt;
    void *P, *X;         // the seed's p and x (stored basis) or those of every shift
    z64 *spart;          // partials of the dotting stencil
    z64 *vpart;          // partials of the seed update (2 per block)
    MsHist *hist;        // scalar history (stored-basis form), hist_cap iterations
    int hist_cap;
    int pad;
    int64_t n;
};

__device__ __forceinline__ z64 cdiv(z64 a, z64 b)
{
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

__device__ __forceinline__ bool finite(z64 a) { return isfinite(a.r) && isfinite(a.i); }

// one block per problem
__global__ void __launch_bounds__(256) ms_alpha_kernel(const MsVec *vl, const int *list)
{
    const MsVec &d = vl[list[blockIdx.x]];
    MsState *S = d.S;
    if (S->h.done) return;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < d.nst_part; i += blockDim.x) {
        re += d.spart[i].r;
        im += d.spart[i].i;
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

// one block per problem; nb = blocks of the seed update that wrote vpart
__global__ void __launch_bounds__(256) ms_beta_kernel(const MsVec *vl, const int *list, int nb)
{
    const MsVec &d = vl[list[blockIdx.x]];
    MsState *S = d.S;
    if (S->h.done) {
        if (threadIdx.x == 0) S->h.go = 0;
        return;
    }
    const int k = S->h.iter;  // this iteration (read before thread 0 advances it)
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        a += d.vpart[2 * i].r;
        b += d.vpart[2 * i].i;
        c += d.vpart[2 * i + 1].r;
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
        S->h.go = bad_sh ? 0 : 1;
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
    MsHist *hk = (d.hist && k < d.hist_cap) ? d.hist + (int64_t)k * S->h.nshift : nullptr;
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

// vectors are in device memory; the pointers come from device-side descriptors, so the
// global address space is stated (global rather than flat instructions)
template <typename T> __device__ __forceinline__ z64 ldz(const T *p, int64_t i)
{
    T v = ((const SGN_GLOBAL T *)p)[i];
    return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stz(double2 *p, int64_t i, z64 v)
{
    ((SGN_GLOBAL double2 *)p)[i] = make_double2(v.r, v.i);
}
__device__ __forceinline__ void stz(float2 *p, int64_t i, z64 v)
{
    ((SGN_GLOBAL float2 *)p)[i] = make_float2((float)v.r, (float)v.i);
}
// Non-temporal forms for the solutions x, read and written once per iteration: they keep this
// stream from evicting the links and the vectors the next kernels read.
typedef float ms_nt_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ z64 ldz_nt(const double2 *p, int64_t i)
{
    const nt_d2 v = __builtin_nontemporal_load((const SGN_GLOBAL nt_d2 *)p + i);
    return {v.x, v.y};
}
__device__ __forceinline__ z64 ldz_nt(const float2 *p, int64_t i)
{
    const ms_nt_f2 v = __builtin_nontemporal_load((const SGN_GLOBAL ms_nt_f2 *)p + i);
    return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stz_nt(double2 *p, int64_t i, z64 v)
{
    __builtin_nontemporal_store(nt_d2{v.r, v.i}, (SGN_GLOBAL nt_d2 *)p + i);
}
__device__ __forceinline__ void stz_nt(float2 *p, int64_t i, z64 v)
{
    __builtin_nontemporal_store(ms_nt_f2{(float)v.r, (float)v.i}, (SGN_GLOBAL ms_nt_f2 *)p + i);
}

// r_{k+1} = r_k - alpha q, r~ -= conj(alpha) q~, with partials of r~^H r_{k+1}
// and ||r_{k+1}||^2.  Per-shift form: in place.  Stored-basis form: from slot k
// (or the replacement residual) into slot k+1.
template <typename R>
__global__ void __launch_bounds__(256) ms_seed_update(const MsVec *vl, const int *list)
{
    using T = typename VecT<R>::t;
    const MsVec &d = vl[list[blockIdx.y]];
    const MsState *S = d.S;
    if (S->h.done) return;
    const int k = S->h.iter;
    const T *r_in;
    T *r_out;
    if (!d.slots) {
        r_out = static_cast<T *>(d.r);
        r_in = r_out;
    } else {
        r_in = static_cast<const T *>(k == d.temp_iter ? d.r : d.slots[k]);
        r_out = static_cast<T *>(d.slots[k + 1]);
    }
    T *rt = static_cast<T *>(d.rt);
    const T *q = static_cast<const T *>(d.q), *qt = static_cast<const T *>(d.qt);
    const int64_t n = d.n;
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
        const z64 dd = cmulc(tv, rv);
        a += dd.r;
        b += dd.i;
        c += norm2(rv);
    }
    __shared__ double lds[12];
    double v[3] = {a, b, c};
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        d.vpart[2 * blockIdx.x] = {v[0], v[1]};
        d.vpart[2 * blockIdx.x + 1] = {v[2], 0.0};
    }
}

// Per-shift form: p_i = zeta_i r + beta_i p_i and x_i += alpha_i p_i (old p_i)
// for every active shift; p~ = r~ + conj(beta) p~.
template <typename R, typename XT>
__global__ void __launch_bounds__(256) ms_shift_update(const MsVec *vl, const int *list,
                                                       unsigned long long *byte_counter)
{
    using T = typename VecT<R>::t;
    const MsVec &d = vl[list[blockIdx.y]];
    const MsState *S = d.S;
    if (S->h.breakdown || !S->h.go) return;
    __shared__ z64 al_s[kS], be_s[kS], ze_s[kS];
    __shared__ int act_s[kS];
    const int nsh = S->h.nshift;
    for (int i = threadIdx.x; i < nsh; i += blockDim.x) {
        act_s[i] = S->act[i];
        al_s[i] = S->alpha_i[i];
        be_s[i] = S->beta_i[i];
        ze_s[i] = S->zeta[i];
    }
    __syncthreads();
    const int64_t n = d.n;
    if (byte_counter && blockIdx.x == 0 && threadIdx.x == 0) {  // algorithmic bytes (profiling)
        unsigned long long na = 0;
        for (int i = 0; i < nsh; ++i) na += act_s[i] ? 1 : 0;
        const unsigned long long eb = sizeof(T), xb = sizeof(XT);
        atomicAdd(byte_counter, (unsigned long long)n * (4ull * eb + na * 2ull * eb + na * 2ull * xb));
    }
    T *P = static_cast<T *>(d.P), *pt = static_cast<T *>(d.pt);
    XT *X = static_cast<XT *>(d.X);
    const T *r = static_cast<const T *>(d.r), *rt = static_cast<const T *>(d.rt);
    const z64 bc = conj(S->h.beta);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 rv = ldz(r, e);
        for (int i = 0; i < nsh; ++i) {
            if (!act_s[i]) continue;
            T *Pi = P + (int64_t)i * n;
            XT *Xi = X + (int64_t)i * n;
            const z64 p = ldz(Pi, e);
            stz_nt(Xi, e, ldz_nt(Xi, e) + al_s[i] * p);
            stz(Pi, e, ze_s[i] * rv + be_s[i] * p);
        }
        stz(pt, e, ldz(rt, e) + bc * ldz(pt, e));
    }
}

// Stored-basis form: only the seed keeps vectors,
//   x_seed += alpha p_seed;  p_seed = r_{k+1} + beta p_seed;  p~ = r~ + conj(beta) p~
// (zeta = 1 and alpha_i = alpha, beta_i = beta for the seed; the values are
// taken from the shift arrays all the same).
template <typename R, typename XT>
__global__ void __launch_bounds__(256) ms_seed_xp_update(const MsVec *vl, const int *list,
                                                         unsigned long long *byte_counter)
{
    using T = typename VecT<R>::t;
    const MsVec &d = vl[list[blockIdx.y]];
    const MsState *S = d.S;
    if (S->h.breakdown || !S->h.go) return;
    const int seed = S->h.seed;
    const z64 al = S->alpha_i[seed], be = S->beta_i[seed], ze = S->zeta[seed], bc = conj(S->h.beta);
    const int64_t n = d.n;
    if (byte_counter && blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd(byte_counter, (unsigned long long)n * (6ull * sizeof(T) + 2ull * sizeof(XT)));
    T *P = static_cast<T *>(d.P), *pt = static_cast<T *>(d.pt);
    XT *X = static_cast<XT *>(d.X);
    const T *r = static_cast<const T *>(d.slots[S->h.iter]), *rt = static_cast<const T *>(d.rt);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const z64 p = ldz(P, e);
        stz_nt(X, e, ldz_nt(X, e) + al * p);
        stz(P, e, ze * ldz(r, e) + be * p);
        stz(pt, e, ldz(rt, e) + bc * ldz(pt, e));
    }
}

// out (+)= sum_j coef_j v_j over up to kLiftChunk stored vectors, FP64 or FP32 each.
// out and FP64 vectors use the [12][S] double2 layout, FP32 vectors the [6][S]
// float4 layout (chunk c holds components 2c and 2c+1); a thread takes one
// component pair of one site, so every load is a full coalesced row.
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
    const int64_t np = (int64_t)6 * Sst;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(p / Sst), st = (int)(p - (int64_t)c2 * Sst);
        const int64_t e0 = (int64_t)(2 * c2) * Sst + st, e1 = e0 + Sst;
        z64 a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
        if (accumulate) {
            const double2 o0 = out[e0], o1 = out[e1];
            a0 = {o0.x, o0.y};
            a1 = {o1.x, o1.y};
        }
        for (int j = 0; j < K; ++j) {
            const z64 c = cf[j];
            if (c.r == 0.0 && c.i == 0.0) continue;  // uniform
            z64 v0, v1;
            if (sl[j].f32) {
                const float4 t = static_cast<const float4 *>(sl[j].p)[p];
                v0 = {(double)t.x, (double)t.y};
                v1 = {(double)t.z, (double)t.w};
            } else {
                const double2 *v = static_cast<const double2 *>(sl[j].p);
                const double2 t0 = v[e0], t1 = v[e1];
                v0 = {t0.x, t0.y};
                v1 = {t1.x, t1.y};
            }
            a0 = a0 + c * v0;
            a1 = a1 + c * v1;
        }
        out[e0] = make_double2(a0.r, a0.i);
        out[e1] = make_double2(a1.r, a1.i);
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

// Host state of one problem of a multishift_solve call.
struct MsProblem {
    const sgn_problem *pb = nullptr;
    Lattice *lat = nullptr;
    sgn_stats *st = nullptr;
    int64_t V = 0, Sst = 0, n = 0, nc = 0;
    size_t b64 = 0, b32 = 0, c64 = 0;
    bool want_shifts = false, explicit_mode = false;
    int slot_cap = 0;
    Span y{}, r{}, rt{}, pt{}, q{}, qt{}, tmp{}, tmpt{}, X{}, P{};
    Span r32{}, rt32{}, pt32{}, q32{}, qt32{}, tmp32{}, tmpt32{}, P32{}, Xlo{};
    Span rcan{};
    MsHist *hist = nullptr;
    MsState *S = nullptr;
    z64 *spart = nullptr, *vpart = nullptr;
    void **slot_table = nullptr;  // device, slot_cap + 1 entries
    std::vector<void *> slots;    // host copy of the slot table
    std::vector<char> slot_f32;   // precision of each stored slot
    int temp_iter = -1;
    std::unique_ptr<DevMem> xp64, xp32;  // per-shift vectors after leaving the stored-basis form
    std::unique_ptr<DevMem> defl_coef;   // m coefficients L^H v of the deflation projection
    OpSpec opA, opAh;
    double ynorm = 0.0;
    int phase = 0, launched = 0, reliable_updates = 0;
    bool active = false;
    sgn_status result = SGN_OK;
    MsHead hh{};
    double kry_ms = 0.0;
};

class MultishiftBatch {
  public:
    MultishiftBatch(const sgn_problem *pb, int nprob, const sgn_rational &rf, const sgn_ms_opts &o,
                    sgn_stats *stats, hipStream_t s);
    ~MultishiftBatch()
    {
        if (gexec_) (void)hipGraphExecDestroy(gexec_);
        if (dheads_) (void)hipFree(dheads_);
        if (hheads_) (void)hipHostFree(hheads_);
    }
    MultishiftBatch(const MultishiftBatch &) = delete;
    MultishiftBatch &operator=(const MultishiftBatch &) = delete;
    sgn_status run();

  private:
    std::vector<MsProblem> pr_;
    const sgn_rational &rf_;
    const sgn_ms_opts &o_;
    hipStream_t s_;
    Context *ctx_ = nullptr;
    int ns_ = 0, seed_ = 0, maxiter_ = 0, poll_ = 1;
    double s1_ = 0.0, c2_ = 0.0;
    bool mixed_ = false;
    std::chrono::steady_clock::time_point t_start_;
    MsVec *dvec_ = nullptr;  // device descriptors, one per problem
    // the heads read after each chunk: the problems' state pointers and a gather buffer (device),
    // and their pinned host mirror (one copy per chunk)
    char *dheads_ = nullptr;
    MsHead *hheads_ = nullptr;
    int *dlist_ = nullptr;   // device problem lists: [3 phases][2 forms][nprob]
    std::vector<MsVec> hvec_;
    std::vector<int> lists_[3][2];  // active problems per phase and form (0 stored basis, 1 per-shift)
    StencilBatch stb_[3][4];        // per phase, the four stencil steps of an iteration
    bool dirty_ = true;             // lists and stencil batches need rebuilding
    bool dirty_vec_ = false;        // only the descriptors changed
    std::map<size_t, size_t> pool_next_;  // next unused pooled slot per vector size in this call
    hipGraphExec_t gexec_ = nullptr;       // captured chunk of poll_ iterations (valid until the next rebuild)
    bool use_graph_ = false;

    void setup(MsProblem &p);
    void rebuild();
    void fill_vec(int k);
    void iterate(int count);               // launches + host bookkeeping of count iterations
    void launch_iterations(int count, hipStream_t strm);
    void drop_graph()
    {
        if (gexec_) SGN_HIP(hipGraphExecDestroy(gexec_));
        gexec_ = nullptr;
    }
    void *slot_ptr(const MsProblem &p, int j) const { return p.slots[(size_t)j]; }
    bool ensure_slots(MsProblem &p, int upto);
    void flush(MsProblem &p);
    void reliable_update(MsProblem &p);
    void project_out(MsProblem &p, void *v);
    void switch_to_f32(MsProblem &p);
    void to_explicit(MsProblem &p);
    void lift(MsProblem &p, const std::vector<z64> &coef, void *out, bool accumulate);
    std::vector<MsHist> history(const MsProblem &p, int k);
    void finish(MsProblem &p);
    double shift_residual(MsProblem &p, int i, const void *xi, void *out);
    int refine(MsProblem &p, int i, void *xi, DevMem &work, int *matvecs);
    void read_heads();
    sgn_prec prec_of(int phase) const
    {
        return phase == 0 ? SGN_PREC_F64 : (phase == 1 ? SGN_PREC_F32 : SGN_PREC_F32_H16);
    }
    void *pseed(const MsProblem &p) const
    {
        const size_t off = p.explicit_mode ? (size_t)seed_ : 0;
        return p.phase >= 1 ? (void *)(p.P32.as<char>() + off * p.b32) : (void *)(p.P.as<char>() + off * p.b64);
    }
};

MultishiftBatch::MultishiftBatch(const sgn_problem *pb, int nprob, const sgn_rational &rf, const sgn_ms_opts &o,
                                 sgn_stats *stats, hipStream_t s)
    : rf_(rf), o_(o), s_(s)
{
    t_start_ = std::chrono::steady_clock::now();
    ns_ = rf.s;
    mixed_ = o.prec != SGN_PREC_F64;
    c2_ = rf.c * rf.c;
    for (int i = 1; i < ns_; ++i)
        if (std::abs(rf.sigma[i]) < std::abs(rf.sigma[seed_])) seed_ = i;
    s1_ = rf.sigma[seed_];
    maxiter_ = o.maxiter > 0 ? o.maxiter : 10000;
    use_graph_ = o.graph >= 0;
    pr_.resize(nprob);
    double basis_bytes_per_iter = 0.0;
    int64_t vtot = 0;
    for (int k = 0; k < nprob; ++k) {
        MsProblem &p = pr_[k];
        p.pb = &pb[k];
        p.lat = as_lattice(pb[k].lat);
        p.st = stats ? &stats[k] : nullptr;
        p.V = p.lat->V;
        p.Sst = p.lat->S;
        p.n = 12 * p.Sst;
        p.nc = 12 * p.V;
        p.b64 = (size_t)p.n * 16;
        p.b32 = (size_t)p.n * 8;
        p.c64 = (size_t)p.nc * 16;
        p.want_shifts = pb[k].x_shift != nullptr || o.verify;
        vtot += p.V;
        if (!p.want_shifts) basis_bytes_per_iter += (double)p.b64;
        if (!ctx_) ctx_ = p.lat->ctx;
        SGN_REQUIRE(p.lat->ctx == ctx_, "multishift_solve: all lattices must share one context");
    }
    SGN_HIP(hipSetDevice(ctx_->device));
    // iterations between host polls: about 200k sites' worth of stencil work per poll, at least 4
    poll_ = o.poll > 0 ? o.poll : (int)std::min<int64_t>(16, std::max<int64_t>(4, (200000 + vtot - 1) / vtot));
    // stored-basis budget: slots per problem
    int cap = 0;
    if (o.basis_slots > 0) {
        cap = o.basis_slots;
    } else if (o.basis_slots == 0 && basis_bytes_per_iter > 0) {
        size_t fr = 0, tot = 0;
        SGN_HIP(hipMemGetInfo(&fr, &tot));
        double held = 0.0;
        for (auto &kv : ctx_->basis_pools) held += (double)kv.first * kv.second.size();
        cap = (int)std::min<double>(1e9, 0.5 * ((double)fr + held) / basis_bytes_per_iter);
    }
    cap = std::min(cap, maxiter_);

    // workspace carved from the context's arena (256-byte aligned pieces)
    auto rs = [](size_t bytes) { return (bytes + 255) / 256 * 256; };
    auto pieces = [&](const MsProblem &p, auto &&take) {
        const size_t np0 = p.explicit_mode ? ns_ : 1;
        const size_t b64 = p.b64, b32 = mixed_ ? p.b32 : 0;
        for (int i = 0; i < 8; ++i) take(b64);           // y r rt pt q qt tmp tmpt
        take(np0 * b64);                                 // X
        take(np0 * b64);                                 // P
        for (int i = 0; i < 7; ++i) take(b32);           // r32 rt32 pt32 q32 qt32 tmp32 tmpt32
        take(np0 * b32);                                 // P32
        take(np0 * b32);                                 // Xlo
        take(p.explicit_mode ? 0 : (size_t)p.slot_cap * ns_ * sizeof(MsHist));
        take(sizeof(MsState));
        take(sizeof(z64) * (size_t)dslash_blocks(*p.lat));
        take(sizeof(z64) * (2 * (size_t)kVecGrid + 2 * (size_t)vec_blocks(6 * p.Sst)));
        take(sizeof(void *) * ((size_t)p.slot_cap + 1));
        take(p.c64);                                     // rcan
    };
    size_t total = 0;
    for (auto &p : pr_) {
        p.explicit_mode = p.want_shifts || cap < 1;
        p.slot_cap = p.explicit_mode ? 0 : cap;
        pieces(p, [&](size_t b) { total += rs(b); });
    }
    total += rs(sizeof(MsVec) * nprob) + rs(sizeof(int) * 6 * nprob);
    char *arena = static_cast<char *>(ctx_->ensure_arena(total));
    for (auto &p : pr_) {
        std::vector<void *> got;
        pieces(p, [&](size_t b) {
            got.push_back(arena);
            arena += rs(b);
        });
        int g = 0;
        for (Span *sp : {&p.y, &p.r, &p.rt, &p.pt, &p.q, &p.qt, &p.tmp, &p.tmpt, &p.X, &p.P, &p.r32, &p.rt32, &p.pt32,
                         &p.q32, &p.qt32, &p.tmp32, &p.tmpt32, &p.P32, &p.Xlo})
            sp->p = got[g++];
        p.hist = static_cast<MsHist *>(got[g++]);
        p.S = static_cast<MsState *>(got[g++]);
        p.spart = static_cast<z64 *>(got[g++]);
        p.vpart = static_cast<z64 *>(got[g++]);
        p.slot_table = static_cast<void **>(got[g++]);
        p.rcan.p = got[g++];
    }
    dvec_ = reinterpret_cast<MsVec *>(arena);
    arena += rs(sizeof(MsVec) * nprob);
    dlist_ = reinterpret_cast<int *>(arena);
    hvec_.resize(nprob);
}

// x <- x_P, y = c A (I - P) b, initial state and vectors of one problem
void MultishiftBatch::setup(MsProblem &p)
{
    Lattice &lat = *p.lat;
    deflation_prologue(*ctx_, p.pb->defl, p.nc, p.pb->b, p.pb->x, p.rcan.p, nullptr, s_);
    p.opA.mu = p.pb->mu;
    p.opAh.mu = -p.pb->mu;
    pack_spinor(lat, p.rcan.p, p.tmp.p, SGN_PREC_F64, s_);
    {
        Epilogue ep;
        ep.a = rf_.c;
        dslash_launch(lat, SGN_PREC_F64, p.opA, p.tmp.p, p.y.p, ep, s_);
    }
    p.ynorm = norm_sync(*ctx_, p.y.p, p.n, false, s_);
    SGN_REQUIRE(std::isfinite(p.ynorm), "multishift_solve: b contains NaN or Inf");
    if (p.st) {
        *p.st = sgn_stats{};
        p.st->nshift = ns_;
    }
    p.active = p.ynorm != 0.0;  // y = 0: x = x_P
    if (!p.active) return;
    MsState h0{};
    h0.h.rho = {p.ynorm * p.ynorm, 0.0};
    h0.h.alpha_prev = {1.0, 0.0};
    h0.h.beta_prev = {0.0, 0.0};
    h0.h.rnorm = h0.h.rmax = h0.h.ynorm = p.ynorm;
    h0.h.tol = o_.tol;
    h0.h.delta = o_.delta > 0 ? o_.delta : 0.1;
    h0.h.theta32 = mixed_ ? (o_.theta32 > 0 ? o_.theta32 : 1e-3) : 0.0;
    // FP16 links perturb the operator by ~1e-3 relative, so its Krylov vectors leave range(I - P)
    // at that rate and excite the deflated modes, which the bi-Lanczos process never reduces:
    // with LR deflation the schedule stops at FP32
    const bool deflated = p.pb->defl && p.pb->defl->m > 0;
    h0.h.theta16 = (o_.prec == SGN_PREC_F32_H16 && !deflated) ? (o_.theta16 > 0 ? o_.theta16 : 1e-6) : 0.0;
    h0.h.maxiter = maxiter_;
    h0.h.nshift = ns_;
    h0.h.seed = seed_;
    for (int i = 0; i < ns_; ++i) {
        h0.zeta[i] = h0.zeta_prev[i] = {1.0, 0.0};
        h0.tau[i] = s1_ - rf_.sigma[i];
        h0.omega[i] = rf_.omega[i];
        h0.act_next[i] = 1;
        h0.res[i] = p.ynorm;
    }
    SGN_HIP(hipMemcpyAsync(p.S, &h0, sizeof(MsState), hipMemcpyHostToDevice, s_));
    SGN_HIP(hipMemcpyAsync(p.r.p, p.y.p, p.b64, hipMemcpyDeviceToDevice, s_));
    SGN_HIP(hipMemcpyAsync(p.rt.p, p.y.p, p.b64, hipMemcpyDeviceToDevice, s_));
    SGN_HIP(hipMemcpyAsync(p.pt.p, p.y.p, p.b64, hipMemcpyDeviceToDevice, s_));
    const int np0 = p.explicit_mode ? ns_ : 1;
    const int nvb = vec_blocks(p.n);
    hipLaunchKernelGGL(copy_rep_kernel, dim3(nvb), dim3(256), 0, s_, p.y.as<double2>(), p.P.as<double2>(), np0, p.n);
    hipLaunchKernelGGL(fill_kernel<double2>, dim3(nvb), dim3(256), 0, s_, p.X.as<double2>(), make_double2(0, 0),
                       (int64_t)np0 * p.n);
    SGN_HIP(hipGetLastError());
    p.slots.assign(1, p.y.p);  // slot 0 is y itself
    p.slot_f32.assign(1, 0);
    if (!p.explicit_mode) SGN_HIP(hipMemcpyAsync(p.slot_table, p.slots.data(), sizeof(void *), hipMemcpyHostToDevice, s_));
    SGN_HIP(hipStreamSynchronize(s_));  // h0 and the slot table entry leave scope
}

// slots 1..upto exist (taken from the context's pool of vectors of this size)
bool MultishiftBatch::ensure_slots(MsProblem &p, int upto)
{
    if (upto > p.slot_cap) return false;
    if ((int)p.slots.size() > upto) return true;
    auto &pool = ctx_->basis_pools[p.b64];
    size_t &nx = pool_next_[p.b64];
    const size_t first = p.slots.size();
    while ((int)p.slots.size() <= upto) {
        if (nx == pool.size()) {
            void *b = nullptr;
            if (hipMalloc(&b, p.b64) != hipSuccess) {
                (void)hipGetLastError();
                return false;
            }
            pool.push_back(b);
        }
        p.slots.push_back(pool[nx++]);
    }
    SGN_HIP(hipMemcpy(p.slot_table + first, p.slots.data() + first, sizeof(void *) * (p.slots.size() - first),
                      hipMemcpyHostToDevice));
    return true;
}

void MultishiftBatch::fill_vec(int k)
{
    MsProblem &p = pr_[k];
    MsVec &v = hvec_[k];
    const int nst_part = v.nst_part;  // set by rebuild() from the stencil batch
    v = MsVec{};
    v.nst_part = nst_part;
    v.S = p.S;
    v.n = p.n;
    v.spart = p.spart;
    v.vpart = p.vpart;
    const bool lo = p.phase >= 1;
    v.r = lo ? p.r32.p : p.r.p;
    v.slots = p.explicit_mode ? nullptr : p.slot_table;
    v.temp_iter = p.temp_iter;
    v.rt = lo ? p.rt32.p : p.rt.p;
    v.q = lo ? p.q32.p : p.q.p;
    v.qt = lo ? p.qt32.p : p.qt.p;
    v.pt = lo ? p.pt32.p : p.pt.p;
    v.P = lo ? p.P32.p : p.P.p;
    v.X = lo ? p.Xlo.p : p.X.p;
    v.hist = p.explicit_mode ? nullptr : p.hist;
    v.hist_cap = p.explicit_mode ? 0 : p.slot_cap;
}

// descriptors, problem lists and stencil batches for the current phases and forms
void MultishiftBatch::rebuild()
{
    drop_graph();
    const int np = (int)pr_.size();
    for (auto &l : lists_)
        for (auto &m : l) m.clear();
    std::vector<StencilJob> jobs[3][4];
    std::vector<int> job_owner[3];
    for (int k = 0; k < np; ++k) {
        MsProblem &p = pr_[k];
        fill_vec(k);
        if (!p.active) continue;
        const MsVec &v = hvec_[k];
        lists_[p.phase][p.explicit_mode ? 1 : 0].push_back(k);
        const bool lo = p.phase >= 1;
        void *ps = pseed(p);
        void *vtmp = lo ? p.tmp32.p : p.tmp.p, *vtmpt = lo ? p.tmpt32.p : p.tmpt.p;
        StencilJob j1{p.lat, p.opA, ps, vtmp, Epilogue{}};
        StencilJob j2{p.lat, p.opA, vtmp, v.q, Epilogue{}};
        j2.ep.a = c2_;
        j2.ep.z = ps;
        j2.ep.b = {-s1_, 0.0};
        j2.ep.w = v.pt;
        j2.ep.partials = p.spart;
        StencilJob j3{p.lat, p.opAh, v.pt, vtmpt, Epilogue{}};
        StencilJob j4{p.lat, p.opAh, vtmpt, v.qt, Epilogue{}};
        j4.ep.a = c2_;
        j4.ep.z = v.pt;
        j4.ep.b = {-s1_, 0.0};
        jobs[p.phase][0].push_back(j1);
        jobs[p.phase][1].push_back(j2);
        jobs[p.phase][2].push_back(j3);
        jobs[p.phase][3].push_back(j4);
        job_owner[p.phase].push_back(k);
    }
    for (int ph = 0; ph < 3; ++ph) {
        for (int st = 0; st < 4; ++st) stb_[ph][st].prepare(jobs[ph][st], prec_of(ph));
        for (size_t j = 0; j < job_owner[ph].size(); ++j) hvec_[job_owner[ph][j]].nst_part = stb_[ph][1].blocks(j);
    }
    SGN_HIP(hipMemcpy(dvec_, hvec_.data(), sizeof(MsVec) * np, hipMemcpyHostToDevice));
    std::vector<int> hl(6 * (size_t)np, 0);
    for (int ph = 0; ph < 3; ++ph)
        for (int form = 0; form < 2; ++form)
            std::copy(lists_[ph][form].begin(), lists_[ph][form].end(), hl.begin() + (size_t)(2 * ph + form) * np);
    SGN_HIP(hipMemcpy(dlist_, hl.data(), sizeof(int) * hl.size(), hipMemcpyHostToDevice));
    dirty_ = dirty_vec_ = false;
}

void MultishiftBatch::iterate(int count)
{
    // the launches only read device-side state, so one capture serves every chunk until the
    // descriptors, lists or stencil batches change
    replay_or_capture(*ctx_, gexec_, use_graph_, s_, [&](hipStream_t strm) { launch_iterations(count, strm); });
    for (int it = 0; it < count; ++it)
        for (auto &p : pr_) {
            if (!p.active) continue;
            ++p.launched;
            if (!p.explicit_mode) {
                if ((int)p.slot_f32.size() <= p.launched) p.slot_f32.resize(p.launched + 1, 0);
                p.slot_f32[p.launched] = p.phase >= 1 ? 1 : 0;
            }
        }
}

void MultishiftBatch::launch_iterations(int count, hipStream_t strm)
{
    const int np = (int)pr_.size();
    for (int it = 0; it < count; ++it) {
        for (int ph = 0; ph < 3; ++ph) {
            const int nb = (int)lists_[ph][0].size(), ne = (int)lists_[ph][1].size();
            if (nb + ne == 0) continue;
            for (int st = 0; st < 4; ++st) stb_[ph][st].launch(strm);
            const int *lb = dlist_ + (size_t)(2 * ph) * np, *le = dlist_ + (size_t)(2 * ph + 1) * np;
            const bool lo = ph >= 1;
            if (nb) hipLaunchKernelGGL(ms_alpha_kernel, dim3(nb), dim3(256), 0, strm, dvec_, lb);
            if (ne) hipLaunchKernelGGL(ms_alpha_kernel, dim3(ne), dim3(256), 0, strm, dvec_, le);
            double elems = 0.0;
            for (int form = 0; form < 2; ++form)
                for (int k : lists_[ph][form]) elems += (double)pr_[k].n;
            const double eb = lo ? 8.0 : 16.0;
            int pr = ctx_->prof_start(strm, SGN_K_SEED_UPDATE);
            for (int form = 0; form < 2; ++form) {
                const int cnt = form ? ne : nb;
                if (!cnt) continue;
                const int *l = form ? le : lb;
                if (lo)
                    hipLaunchKernelGGL(ms_seed_update<float>, dim3(kVecGrid, cnt), dim3(256), 0, strm, dvec_, l);
                else
                    hipLaunchKernelGGL(ms_seed_update<double>, dim3(kVecGrid, cnt), dim3(256), 0, strm, dvec_, l);
            }
            ctx_->prof_stop(pr, strm, SGN_K_SEED_UPDATE, 6.0 * eb * elems, 40.0 * elems);
            if (nb) hipLaunchKernelGGL(ms_beta_kernel, dim3(nb), dim3(256), 0, strm, dvec_, lb, kVecGrid);
            if (ne) hipLaunchKernelGGL(ms_beta_kernel, dim3(ne), dim3(256), 0, strm, dvec_, le, kVecGrid);
            pr = ctx_->prof_start(strm, SGN_K_SHIFT_UPDATE);
            unsigned long long *bc = pr >= 0 ? ctx_->byte_counter : nullptr;  // bytes of sampled launches only
            if (nb) {
                if (lo)
                    hipLaunchKernelGGL((ms_seed_xp_update<float, float2>), dim3(kVecGrid, nb), dim3(256), 0, strm,
                                       dvec_, lb, bc);
                else
                    hipLaunchKernelGGL((ms_seed_xp_update<double, double2>), dim3(kVecGrid, nb), dim3(256), 0, strm,
                                       dvec_, lb, bc);
            }
            if (ne) {
                if (lo)
                    hipLaunchKernelGGL((ms_shift_update<float, float2>), dim3(kVecGrid, ne), dim3(256), 0, strm, dvec_,
                                       le, bc);
                else
                    hipLaunchKernelGGL((ms_shift_update<double, double2>), dim3(kVecGrid, ne), dim3(256), 0, strm,
                                       dvec_, le, bc);
            }
            ctx_->prof_stop(pr, strm, SGN_K_SHIFT_UPDATE, 0.0, 0.0, true);
        }
    }
    SGN_HIP(hipGetLastError());
}

void MultishiftBatch::flush(MsProblem &p)
{
    hipLaunchKernelGGL(ms_flush_kernel, dim3(vec_blocks(6 * p.Sst)), dim3(256), 0, s_, p.X.as<double2>(),
                       p.Xlo.as<float4>(), p.explicit_mode ? ns_ : 1, (int)p.Sst);
}

// v = (I - P) v for an FP64 vector in the internal layout (canonical round trip),
// P = R L^H the LR-deflation projector of the problem; no-op without deflation.
void MultishiftBatch::project_out(MsProblem &p, void *v)
{
    const sgn_deflation *defl = p.pb->defl;
    if (!defl || defl->m <= 0) return;
    if (!p.defl_coef) p.defl_coef = std::make_unique<DevMem>(sizeof(z64) * defl->m);
    unpack_spinor(*p.lat, v, p.rcan.p, SGN_PREC_F64, s_);
    deflate_dots(defl->L, defl->m, p.rcan.p, p.nc, p.defl_coef->as<z64>(), *ctx_, s_);
    deflate_combine(p.rcan.p, {1.0, 0.0}, {-1.0, 0.0}, defl->R, defl->m, p.defl_coef->as<z64>(), nullptr, p.nc, s_);
    pack_spinor(*p.lat, p.rcan.p, v, SGN_PREC_F64, s_);
}

void MultishiftBatch::reliable_update(MsProblem &p)
{
    flush(p);
    double2 *xs = p.X.as<double2>() + (p.explicit_mode ? (size_t)seed_ * p.n : 0);
    // the exact solution lies in range(I - P) (y does and P commutes with A); the
    // reduced-precision iterations leave rounding components along the deflated
    // eigenvectors that the bi-Lanczos process never reduces (its shadow space is
    // orthogonal to them), so they are removed here, the projection step of the
    // restarted methods applied at every true-residual recomputation
    project_out(p, xs);
    dslash_launch(*p.lat, SGN_PREC_F64, p.opA, xs, p.tmp.p, Epilogue{}, s_);
    Epilogue ep;
    ep.a = -c2_;
    ep.z = xs;
    ep.b = {s1_, 0.0};
    dslash_launch(*p.lat, SGN_PREC_F64, p.opA, p.tmp.p, p.q.p, ep, s_);  // q = -c^2 A A x + sigma x
    const int nvbp = vec_blocks(6 * p.Sst);
    z64 *part = p.vpart + 2 * kVecGrid;
    hipLaunchKernelGGL(ms_reliable_kernel, dim3(nvbp), dim3(256), 0, s_, p.y.as<double2>(), p.q.as<double2>(),
                       p.r32.as<float4>(), p.rt32.as<float4>(), (int)p.Sst, part);
    hipLaunchKernelGGL(ms_reliable_coef, dim3(1), dim3(256), 0, s_, part, nvbp, p.S);
    SGN_HIP(hipGetLastError());
    if (!p.explicit_mode) {  // the next seed update starts from r32 instead of its slot
        p.temp_iter = p.launched;
        dirty_vec_ = true;
    }
    ++p.reliable_updates;
}

void MultishiftBatch::switch_to_f32(MsProblem &p)
{
    convert_64_to_32(p.explicit_mode ? p.r.p : slot_ptr(p, p.launched), p.r32.p, p.Sst, s_);
    if (!p.explicit_mode) p.temp_iter = p.launched;
    convert_64_to_32(p.rt.p, p.rt32.p, p.Sst, s_);
    convert_64_to_32(p.pt.p, p.pt32.p, p.Sst, s_);
    const int np0 = p.explicit_mode ? ns_ : 1;
    for (int i = 0; i < np0; ++i)
        convert_64_to_32(p.P.as<char>() + (size_t)i * p.b64, p.P32.as<char>() + (size_t)i * p.b32, p.Sst, s_);
    hipLaunchKernelGGL(fill_kernel<float2>, dim3(vec_blocks(p.n)), dim3(256), 0, s_, p.Xlo.as<float2>(),
                       make_float2(0, 0), (int64_t)np0 * p.n);
    SGN_HIP(hipGetLastError());
    dirty_ = true;
}

// out (+)= sum_j coef[j] slot_j over slots 0..K-1
void MultishiftBatch::lift(MsProblem &p, const std::vector<z64> &coef, void *out, bool accumulate)
{
    const int K = (int)coef.size();
    std::vector<LiftSlot> hs(K);
    double bytes = accumulate ? 2.0 * p.b64 : (double)p.b64;
    for (int j = 0; j < K; ++j) {
        hs[j] = LiftSlot{slot_ptr(p, j), p.slot_f32[j], 0};
        bytes += (coef[j].r != 0.0 || coef[j].i != 0.0) ? (p.slot_f32[j] ? (double)p.b32 : (double)p.b64) : 0.0;
    }
    DevMem dsl(sizeof(LiftSlot) * std::max(K, 1)), dcf(sizeof(z64) * std::max(K, 1));
    if (K) {
        SGN_HIP(hipMemcpy(dsl.p, hs.data(), sizeof(LiftSlot) * K, hipMemcpyHostToDevice));
        SGN_HIP(hipMemcpy(dcf.p, coef.data(), sizeof(z64) * K, hipMemcpyHostToDevice));
    }
    const int pr = ctx_->prof_start(s_, SGN_K_LIFT);
    const int nvb = vec_blocks(p.n);
    if (K == 0 && !accumulate)
        hipLaunchKernelGGL(fill_kernel<double2>, dim3(nvb), dim3(256), 0, s_, static_cast<double2 *>(out),
                           make_double2(0, 0), p.n);
    for (int j0 = 0; j0 < K; j0 += kLiftChunk) {
        const int kk = std::min(kLiftChunk, K - j0);
        hipLaunchKernelGGL(ms_lift_kernel, dim3(vec_blocks(6 * p.Sst)), dim3(256), 0, s_, dsl.as<LiftSlot>() + j0,
                           dcf.as<z64>() + j0, kk, (int)p.Sst, static_cast<double2 *>(out), (accumulate || j0 > 0) ? 1 : 0);
    }
    SGN_HIP(hipGetLastError());
    ctx_->prof_stop(pr, s_, SGN_K_LIFT, bytes, 8.0 * p.n * K);
    SGN_HIP(hipStreamSynchronize(s_));  // dsl, dcf go out of scope
}

std::vector<MsHist> MultishiftBatch::history(const MsProblem &p, int k)
{
    std::vector<MsHist> H((size_t)k * ns_);
    if (k > 0) SGN_HIP(hipMemcpy(H.data(), p.hist, sizeof(MsHist) * H.size(), hipMemcpyDeviceToHost));
    return H;
}

// Turn the stored basis into explicit p_i, x_i at iteration k = launched
// (all launched iterations have run) and continue with per-shift vectors.
void MultishiftBatch::to_explicit(MsProblem &p)
{
    const int k = p.launched;
    const std::vector<MsHist> H = history(p, k);
    p.xp64 = std::make_unique<DevMem>(2 * (size_t)ns_ * p.b64);
    if (mixed_) p.xp32 = std::make_unique<DevMem>(2 * (size_t)ns_ * p.b32);
    Span Xn{p.xp64->p}, Pn{p.xp64->as<char>() + (size_t)ns_ * p.b64};
    Span Xlon{mixed_ ? p.xp32->p : nullptr}, P32n{mixed_ ? p.xp32->as<char>() + (size_t)ns_ * p.b32 : nullptr};
    if (p.phase >= 1) flush(p);
    std::vector<z64> cj, aj;
    for (int i = 0; i < ns_; ++i) {
        char *xi = Xn.as<char>() + (size_t)i * p.b64, *pi = Pn.as<char>() + (size_t)i * p.b64;
        if (i == seed_) {
            SGN_HIP(hipMemcpyAsync(xi, p.X.p, p.b64, hipMemcpyDeviceToDevice, s_));
            if (p.phase >= 1)
                SGN_HIP(hipMemcpyAsync(P32n.as<char>() + (size_t)i * p.b32, p.P32.p, p.b32, hipMemcpyDeviceToDevice, s_));
            else
                SGN_HIP(hipMemcpyAsync(pi, p.P.p, p.b64, hipMemcpyDeviceToDevice, s_));
            continue;
        }
        basis_coefficients(H, ns_, k, i, &cj, &aj);
        lift(p, cj, xi, false);
        lift(p, aj, pi, false);
        if (p.phase >= 1) convert_64_to_32(pi, P32n.as<char>() + (size_t)i * p.b32, p.Sst, s_);
    }
    if (mixed_)
        hipLaunchKernelGGL(fill_kernel<float2>, dim3(vec_blocks(p.n)), dim3(256), 0, s_, Xlon.as<float2>(),
                           make_float2(0, 0), (int64_t)ns_ * p.n);
    // the per-shift form keeps the current residual in r (FP64) or r32
    void *cur = (p.temp_iter == k) ? (p.phase >= 1 ? p.r32.p : p.r.p) : slot_ptr(p, k);
    if (p.phase >= 1) {
        if (cur != p.r32.p) SGN_HIP(hipMemcpyAsync(p.r32.p, cur, p.b32, hipMemcpyDeviceToDevice, s_));
    } else {
        if (cur != p.r.p) SGN_HIP(hipMemcpyAsync(p.r.p, cur, p.b64, hipMemcpyDeviceToDevice, s_));
    }
    SGN_HIP(hipStreamSynchronize(s_));
    p.X = Xn;
    p.P = Pn;
    p.Xlo = Xlon;
    p.P32 = P32n;
    p.explicit_mode = true;
    dirty_ = true;
}

void MultishiftBatch::read_heads()
{
    const int np = (int)pr_.size();
    if (!dheads_) {
        std::vector<MsState *> sp(np);
        for (int k = 0; k < np; ++k) sp[k] = pr_[k].S;
        if (hipMalloc(&dheads_, (sizeof(MsState *) + sizeof(MsHead)) * np) != hipSuccess) {
            dheads_ = nullptr;
            throw Failure{SGN_ERR_NOMEM, "multishift_solve: batch heads"};
        }
        SGN_HIP(hipMemcpy(dheads_, sp.data(), sizeof(MsState *) * np, hipMemcpyHostToDevice));
        SGN_HIP(hipHostMalloc(reinterpret_cast<void **>(&hheads_), sizeof(MsHead) * np));
    }
    MsState *const *dsp = reinterpret_cast<MsState *const *>(dheads_);
    MsHead *dh = reinterpret_cast<MsHead *>(dheads_ + sizeof(MsState *) * np);
    hipLaunchKernelGGL(ms_gather_heads, dim3(np), dim3(64), 0, s_, dsp, dh);
    SGN_HIP(hipGetLastError());
    SGN_HIP(hipMemcpyAsync(hheads_, dh, sizeof(MsHead) * np, hipMemcpyDeviceToHost, s_));
    SGN_HIP(hipStreamSynchronize(s_));
    for (int k = 0; k < np; ++k)
        if (pr_[k].active) {
            pr_[k].hh = hheads_[k];
            pr_[k].launched = pr_[k].hh.iter;
        }
}

// out = y - (c^2 A^2 - sigma_i) x_i in FP64 (internal layout); returns its norm
double MultishiftBatch::shift_residual(MsProblem &p, int i, const void *xi, void *out)
{
    Lattice &lat = *p.lat;
    dslash_launch(lat, SGN_PREC_F64, p.opA, xi, p.tmp.p, Epilogue{}, s_);
    Epilogue ep;
    ep.a = -c2_;
    ep.z = xi;
    ep.b = {rf_.sigma[i], 0.0};
    dslash_launch(lat, SGN_PREC_F64, p.opA, p.tmp.p, out, ep, s_);
    axpby64({1.0, 0.0}, p.y.p, {1.0, 0.0}, out, p.n, s_);
    return norm_sync(*ctx_, out, p.n, false, s_);
}

// Per-shift FP64 refinement: x_i += e with (c^2 A^2 - sigma_i) e = r_i, r_i (in p.q) the true
// residual of x_i, by FP64 BiCGStab on that one system until ||r|| <= tol ||y|| / 2.  Returns
// the iterations used.
int MultishiftBatch::refine(MsProblem &p, int i, void *xi, DevMem &work, int *matvecs)
{
    return refine_shift64(*p.lat, p.opA, c2_, rf_.sigma[i], p.q.p, xi, 0.5 * o_.tol * p.ynorm, maxiter_, work.p,
                          p.tmp.p, s_, matvecs);
}

// x += sum_i omega_i x_i, outputs and statistics of one problem
void MultishiftBatch::finish(MsProblem &p)
{
    Lattice &lat = *p.lat;
    const int nvb = vec_blocks(p.n);
    // FP64 true residual of every shifted system (the per-shift solutions are explicit when
    // verifying); a system above the tolerance is refined before the combination
    std::vector<double> vres;
    int refine_its = 0, extra_mv = 0;
    if (o_.verify && p.ynorm != 0.0) {
        vres.assign(ns_, 0.0);
        std::unique_ptr<DevMem> work;
        for (int i = 0; i < ns_; ++i) {
            double2 *xi = p.X.as<double2>() + (size_t)i * p.n;
            vres[i] = shift_residual(p, i, xi, p.q.p) / p.ynorm;
            extra_mv += 2;
            if (vres[i] > o_.tol) {
                if (!work) work = std::make_unique<DevMem>(6 * p.b64);
                refine_its += refine(p, i, xi, *work, &extra_mv);
                vres[i] = shift_residual(p, i, xi, p.q.p) / p.ynorm;
                extra_mv += 2;
                if (vres[i] > o_.tol && p.result == SGN_OK) p.result = SGN_ERR_NOT_CONVERGED;
            }
        }
    }
    if (p.ynorm != 0.0) {
        if (p.explicit_mode) {
            DevMem w(sizeof(double) * ns_);
            SGN_HIP(hipMemcpy(w.p, rf_.omega, sizeof(double) * ns_, hipMemcpyHostToDevice));
            hipLaunchKernelGGL(ms_combine_kernel, dim3(nvb), dim3(256), 0, s_, p.X.as<double2>(), w.as<double>(),
                               ns_, p.n, p.tmp.as<double2>());
            SGN_HIP(hipGetLastError());
            SGN_HIP(hipStreamSynchronize(s_));
        } else {
            // omega_seed x_seed + sum_j d_j r_j,  d_j = sum_{i != seed} omega_i c_ij
            const int K = p.launched;
            const std::vector<MsHist> H = history(p, K);
            std::vector<z64> d(K, z64{0.0, 0.0}), cj;
            for (int i = 0; i < ns_; ++i) {
                if (i == seed_) continue;
                basis_coefficients(H, ns_, K, i, &cj, nullptr);
                for (int j = 0; j < K; ++j) d[j] = d[j] + rf_.omega[i] * cj[j];
            }
            scale64({rf_.omega[seed_], 0.0}, p.X.p, p.tmp.p, p.n, s_);
            lift(p, d, p.tmp.p, true);
        }
        project_out(p, p.tmp.p);  // rounding components along the deflated eigenvectors
        unpack_spinor(lat, p.tmp.p, p.rcan.p, SGN_PREC_F64, s_);
        axpby64({1.0, 0.0}, p.rcan.p, {1.0, 0.0}, p.pb->x, p.nc, s_);
    }
    if (p.pb->x_shift)
        for (int i = 0; i < ns_; ++i)
            if (p.pb->x_shift[i]) {
                if (p.ynorm != 0.0)
                    unpack_spinor(lat, p.X.as<char>() + (size_t)i * p.b64, p.pb->x_shift[i], SGN_PREC_F64, s_);
                else
                    SGN_HIP(hipMemsetAsync(p.pb->x_shift[i], 0, p.c64, s_));
            }
    SGN_HIP(hipStreamSynchronize(s_));
    if (!p.st || p.ynorm == 0.0) return;
    sgn_stats *st = p.st;
    MsState hs;
    SGN_HIP(hipMemcpy(&hs, p.S, sizeof(MsState), hipMemcpyDeviceToHost));
    st->iterations = hs.h.iter;
    st->matvecs = 4 * hs.h.iter + 1 + 2 * p.reliable_updates + extra_mv;
    st->reliable_updates = p.reliable_updates;
    st->refine_iterations = refine_its;
    double mx = 0.0;
    for (int i = 0; i < ns_; ++i) {
        st->shift_residual[i] = o_.verify ? vres[i] : hs.res[i] / p.ynorm;
        mx = std::max(mx, st->shift_residual[i]);
    }
    st->residual = mx;
    st->krylov_ms = p.kry_ms;
    st->total_ms = ms_since(t_start_);
}

sgn_status MultishiftBatch::run()
{
    for (auto &p : pr_) setup(p);
    const auto t_kry = std::chrono::steady_clock::now();
    for (;;) {
        bool any = false;
        for (auto &p : pr_) {
            if (!p.active) continue;
            any = true;
            // slots for the next chunk; past the budget the basis becomes per-shift vectors
            if (!p.explicit_mode && !ensure_slots(p, p.launched + poll_)) to_explicit(p);
        }
        if (!any) break;
        if (dirty_) {
            rebuild();
        } else if (dirty_vec_) {
            for (int k = 0; k < (int)pr_.size(); ++k) fill_vec(k);
            SGN_HIP(hipMemcpy(dvec_, hvec_.data(), sizeof(MsVec) * pr_.size(), hipMemcpyHostToDevice));
            dirty_vec_ = false;
        }
        iterate(poll_);
        read_heads();
        for (auto &p : pr_) {
            if (!p.active) continue;
            MsHead &hh = p.hh;
            if (hh.breakdown)
                throw Failure{SGN_ERR_BREAKDOWN, "multishift BiCG breakdown at iteration " + std::to_string(hh.iter)};
            if (hh.done) {
                if (p.phase >= 1) {
                    reliable_update(p);
                    SGN_HIP(hipMemcpyAsync(&hh, &p.S->h, sizeof(MsHead), hipMemcpyDeviceToHost, s_));
                    SGN_HIP(hipStreamSynchronize(s_));
                    if (!hh.done) continue;
                }
                if (hh.iter >= maxiter_ && hh.rnorm > o_.tol * p.ynorm) p.result = SGN_ERR_NOT_CONVERGED;
                if (p.phase >= 1) flush(p);
                p.kry_ms = ms_since(t_kry);
                p.active = false;
                dirty_ = true;
                continue;
            }
            if (mixed_ && hh.want_phase > p.phase) {
                const int zero = 0;
                if (p.phase == 0) {
                    switch_to_f32(p);
                    p.phase = 1;
                    const double rm = hh.rnorm;
                    SGN_HIP(hipMemcpyAsync(&p.S->h.rmax, &rm, sizeof(double), hipMemcpyHostToDevice, s_));
                    SGN_HIP(hipStreamSynchronize(s_));
                } else if (p.phase == 1 && o_.prec == SGN_PREC_F32_H16) {
                    p.phase = 2;
                }
                const int ph = p.phase;
                SGN_HIP(hipMemcpyAsync(&p.S->h.phase, &ph, sizeof(int), hipMemcpyHostToDevice, s_));
                SGN_HIP(hipMemcpyAsync(&p.S->h.want_phase, &zero, sizeof(int), hipMemcpyHostToDevice, s_));
                SGN_HIP(hipStreamSynchronize(s_));
                dirty_ = true;
                continue;
            }
            if (p.phase >= 1 && hh.reliable) reliable_update(p);
        }
    }
    sgn_status worst = SGN_OK;
    for (auto &p : pr_) {
        finish(p);
        if (p.result != SGN_OK && worst == SGN_OK) worst = p.result;
    }
    return worst;
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
        if (nprob == 0) return;
        MultishiftBatch batch(pb, nprob, *rf, *o, stats, static_cast<hipStream_t>(stream));
        worst = batch.run();
    });
    return st != SGN_OK ? st : worst;
}
