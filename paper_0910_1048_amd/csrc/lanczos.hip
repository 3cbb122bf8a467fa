// Direct two-sided Lanczos-LR(m, k): sign(H_W) b = x_P + ||r|| V_k sign(T_k) e_1
// (section "Direct application of the two-sided Lanczos approach"; the
// recurrences (2sided1), (2sided2) with A = H_W(mu), A^H = H_W(-mu)).
//
// Basis vectors are kept unnormalised: v_j = s_j vh_j, w_j = t_j wh_j, with the
// real scale s_j and complex scale t_j in device memory.  No separate scaling
// pass is needed: every kernel that reads a basis vector folds its scale into
// its coefficients, and the lift folds s_j into the coefficients of V_k.
//
// Per step j (all coefficients FP64, computed on the device):
//   stencil  u  = A vh_j,    partials of wh_j^H u       (epilogue-fused dot)
//   finalize alpha_j = conj(t_j) s_j wh_j^H u          (= w_j^H A v_j)
//   stencil  z  = A^H wh_j
//   update   vh_{j+1} = s_j u - alpha_j s_j vh_j - h_{j-1,j} s_{j-1} vh_{j-1}
//            wh_{j+1} = t_j z - conj(alpha_j) t_j wh_j - conj(h_{j,j-1}) t_{j-1} wh_{j-1}
//            partials of ||vh||^2, wh^H vh, ||wh||^2
//   finalize h_{j+1,j} = ||vh_{j+1}||, s_{j+1} = 1/h_{j+1,j},
//            h_{j,j+1} = wh_{j+1}^H v_{j+1},  t_{j+1} = 1/conj(h_{j,j+1})
//
// The second part of the file runs the same recurrence on c^2 H_W^2 for the
// multishift QMR solver (multishift_qmr).
#include <algorithm>
#include <chrono>
#include <complex>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "field_io.h"
#include "launch.h"
#include "small_sign.h"
#include "vec.h"

namespace sgn {

namespace {

// device scalar block of one solve
struct LzScalars {
    z64 *alpha;  // [k]   h_{jj}
    z64 *hsub;   // [k]   h_{j+1,j} (real, stored complex)
    z64 *hsup;   // [k]   h_{j,j+1}
    z64 *sv;     // [k+1] s_j
    z64 *tw;     // [k+1] t_j
    int *flag;   // [k]   breakdown flags
};

__device__ __forceinline__ void lz_alpha_body(const z64 *partials, int nblk, const LzScalars &S, int j)
{
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        re += partials[i].r;
        im += partials[i].i;
    }
    __shared__ double lds[8];
    double v[2] = {re, im};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        const z64 d = {v[0], v[1]};
        S.alpha[j] = S.sv[j].r * cmulc(S.tw[j], d);  // conj(t_j) s_j (wh^H u)
    }
}
__global__ void lz_alpha_kernel(const z64 *partials, int nblk, LzScalars S, int j)
{
    lz_alpha_body(partials, nblk, S, j);
}

__device__ __forceinline__ void lz_step_body(const z64 *partials, int nblk, const LzScalars &S, int j, double tol)
{
    double a = 0.0, br = 0.0, bi = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        a += partials[2 * i].r;
        br += partials[2 * i].i;
        bi += partials[2 * i + 1].r;
        c += partials[2 * i + 1].i;
    }
    __shared__ double lds[16];
    double v[4] = {a, br, bi, c};
    block_sum<4>(v, lds);
    if (threadIdx.x == 0) {
        const double vv = v[0], ww = v[3];
        const z64 wv = {v[1], v[2]};
        const double delta = sqrt(vv);
        const double sn = delta > 0.0 ? 1.0 / delta : 0.0;
        const z64 hsup = sn * wv;
        S.hsub[j] = {delta, 0.0};
        S.hsup[j] = hsup;
        S.sv[j + 1] = {sn, 0.0};
        const double m2 = norm2(hsup);
        S.tw[j + 1] = m2 > 0.0 ? z64{hsup.r / m2, hsup.i / m2} : z64{0.0, 0.0};  // 1/conj(h)
        S.flag[j] = (!(delta > 0.0) || !(sqrt(norm2(wv)) > tol * sqrt(vv * ww))) ? 1 : 0;
    }
}
__global__ void lz_step_kernel(const z64 *partials, int nblk, LzScalars S, int j, double tol)
{
    lz_step_body(partials, nblk, S, j, tol);
}

__device__ __forceinline__ z64 ld2(const double2 *p, int64_t i)
{
    double2 t = p[i];
    return {t.x, t.y};
}

// One thread per pair of complex entries (e0 = 2*c2*V + s, e1 = e0 + V) so that
// the FP32 stencil outputs ([6][V] float4) and FP64 vectors line up.  vc, wc (may be null): second
// FP64 copies of vh_{j+1}, wh_{j+1} (the fixed stencil inputs of a lockstep batch).
template <bool F32>
__device__ __forceinline__ void lz_update_body(const void *u_, const void *z_, const double2 *vj, const double2 *vjm,
                                               const double2 *wj, const double2 *wjm, double2 *vn, double2 *wn,
                                               float4 *vn32, float4 *wn32, double2 *vc, double2 *wc,
                                               const LzScalars &S, int j, int V /* component stride */,
                                               z64 *partials)
{
    // coefficients of the two three-term recurrences
    const double s0 = S.sv[j].r;
    const z64 al = S.alpha[j], t0 = S.tw[j];
    const z64 cu = {s0, 0.0};
    const z64 cv0 = -(s0 * al);
    const z64 cz = t0;
    const z64 cw0 = -(conj(al) * t0);
    z64 cv1 = {0.0, 0.0}, cw1 = {0.0, 0.0};
    if (j > 0) {
        cv1 = -(S.sv[j - 1].r * S.hsup[j - 1]);       // h_{j-1,j} s_{j-1}
        cw1 = -(conj(S.hsub[j - 1]) * S.tw[j - 1]);   // conj(h_{j,j-1}) t_{j-1}
    }
    const int64_t npair = (int64_t)6 * V;
    double a = 0.0, br = 0.0, bi = 0.0, c = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npair; p += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(p / V), s = (int)(p - (int64_t)c2 * V);
        const int64_t e0 = (int64_t)(2 * c2) * V + s, e1 = e0 + V;
        z64 u0, u1, z0, z1;
        if constexpr (F32) {
            float4 uu = static_cast<const float4 *>(u_)[p], zz = static_cast<const float4 *>(z_)[p];
            u0 = {uu.x, uu.y};
            u1 = {uu.z, uu.w};
            z0 = {zz.x, zz.y};
            z1 = {zz.z, zz.w};
        } else {
            u0 = ld2(static_cast<const double2 *>(u_), e0);
            u1 = ld2(static_cast<const double2 *>(u_), e1);
            z0 = ld2(static_cast<const double2 *>(z_), e0);
            z1 = ld2(static_cast<const double2 *>(z_), e1);
        }
        z64 v0 = cu * u0 + cv0 * ld2(vj, e0), v1 = cu * u1 + cv0 * ld2(vj, e1);
        z64 w0 = cz * z0 + cw0 * ld2(wj, e0), w1 = cz * z1 + cw0 * ld2(wj, e1);
        if (j > 0) {
            v0 = v0 + cv1 * ld2(vjm, e0);
            v1 = v1 + cv1 * ld2(vjm, e1);
            w0 = w0 + cw1 * ld2(wjm, e0);
            w1 = w1 + cw1 * ld2(wjm, e1);
        }
        vn[e0] = make_double2(v0.r, v0.i);
        vn[e1] = make_double2(v1.r, v1.i);
        wn[e0] = make_double2(w0.r, w0.i);
        wn[e1] = make_double2(w1.r, w1.i);
        if constexpr (F32) {
            vn32[p] = make_float4((float)v0.r, (float)v0.i, (float)v1.r, (float)v1.i);
            wn32[p] = make_float4((float)w0.r, (float)w0.i, (float)w1.r, (float)w1.i);
        }
        if (vc) {  // uniform
            vc[e0] = make_double2(v0.r, v0.i);
            vc[e1] = make_double2(v1.r, v1.i);
            wc[e0] = make_double2(w0.r, w0.i);
            wc[e1] = make_double2(w1.r, w1.i);
        }
        a += norm2(v0) + norm2(v1);
        const z64 d = cmulc(w0, v0) + cmulc(w1, v1);
        br += d.r;
        bi += d.i;
        c += norm2(w0) + norm2(w1);
    }
    __shared__ double lds[16];
    double v[4] = {a, br, bi, c};
    block_sum<4>(v, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = {v[0], v[1]};
        partials[2 * blockIdx.x + 1] = {v[2], v[3]};
    }
}
template <bool F32>
__global__ void __launch_bounds__(256) lz_update_kernel(const void *u_, const void *z_, const double2 *vj,
                                                        const double2 *vjm, const double2 *wj, const double2 *wjm,
                                                        double2 *vn, double2 *wn, float4 *vn32, float4 *wn32,
                                                        double2 *vc, double2 *wc, LzScalars S, int j, int V,
                                                        z64 *partials)
{
    lz_update_body<F32>(u_, z_, vj, vjm, wj, wjm, vn, wn, vn32, wn32, vc, wc, S, j, V, partials);
}

constexpr int kLiftChunk = 64;

// out[e] (+)= sum_j coef_j vec_j[e] over a table of K <= kLiftChunk FP64 vectors
__global__ void __launch_bounds__(256) basis_lift_kernel(const double2 *const *vecs, const z64 *coef, int K,
                                                         int64_t n, double2 *out, int accumulate)
{
    __shared__ const double2 *vp[kLiftChunk];
    __shared__ z64 cf[kLiftChunk];
    if ((int)threadIdx.x < K) {
        vp[threadIdx.x] = vecs[threadIdx.x];
        cf[threadIdx.x] = coef[threadIdx.x];
    }
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        z64 acc = {0.0, 0.0};
        if (accumulate) acc = ld2(out, e);
        for (int j = 0; j < K; ++j) acc = acc + cf[j] * ld2(vp[j], e);
        out[e] = make_double2(acc.r, acc.i);
    }
}

struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t bytes)
    {
        if (bytes && hipMalloc(&p, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "device workspace"};
    }
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Stored Krylov vectors (FP64, internal layout) taken on demand from the context's pool of
// vectors of this size; the pool keeps them between calls, so memory follows the steps
// actually taken.  At most cap vectors (SGN_ERR_NOMEM beyond, or when allocation fails).
struct PooledBasis {
    Context &ctx;
    size_t bytes, cap;
    const char *who;
    std::vector<void *> slots;
    size_t *shared_next = nullptr;  // bases sharing one pool (a batch): the next unused pool buffer
    PooledBasis(Context &c, size_t b, size_t cap_, const char *w) : ctx(c), bytes(b), cap(cap_), who(w) {}
    void *operator[](int j) const { return slots[j]; }
    void ensure(int upto)  // slots 0 .. upto exist
    {
        auto &pool = ctx.basis_pools[bytes];
        while ((int)slots.size() <= upto) {
            if (slots.size() >= cap)
                throw Failure{SGN_ERR_NOMEM, std::string(who) + ": Krylov basis exceeds its slot budget"};
            const size_t idx = shared_next ? (*shared_next)++ : slots.size();
            if (idx == pool.size()) {
                void *v = nullptr;
                if (hipMalloc(&v, bytes) != hipSuccess) {
                    (void)hipGetLastError();
                    throw Failure{SGN_ERR_NOMEM, std::string(who) + ": Krylov basis does not fit"};
                }
                pool.push_back(v);
            }
            slots.push_back(pool[idx]);
        }
    }
    // out = sum_{j < K} dcoef[j] slot_j; dtab holds the K slot pointers on the device.  The
    // launches are stream-ordered: dcoef and dtab must stay valid until they have run.
    void lift(const z64 *dcoef, const void *const *dtab, int K, int64_t n, void *out, hipStream_t s) const
    {
        for (int j0 = 0; j0 < K; j0 += kLiftChunk) {
            const int kk = std::min(kLiftChunk, K - j0);
            hipLaunchKernelGGL(basis_lift_kernel, dim3(vec_blocks(n)), dim3(256), 0, s,
                               reinterpret_cast<const double2 *const *>(dtab) + j0, dcoef + j0, kk, n,
                               static_cast<double2 *>(out), j0 > 0 ? 1 : 0);
        }
        SGN_HIP(hipGetLastError());
    }
};

}  // namespace

void deflation_prologue(Context &ctx, const sgn_deflation *defl, int64_t n, const void *b, void *x, void *r,
                        void *rt, hipStream_t s, bool check)
{
    const size_t bytes = (size_t)n * 16;
    const int m = (defl && defl->m > 0) ? defl->m : 0;
    if (m == 0) {
        if (r) SGN_HIP(hipMemcpyAsync(r, b, bytes, hipMemcpyDeviceToDevice, s));
        if (rt) SGN_HIP(hipMemcpyAsync(rt, b, bytes, hipMemcpyDeviceToDevice, s));
        if (x) SGN_HIP(hipMemsetAsync(x, 0, bytes, s));
        return;
    }
    SGN_REQUIRE(defl->L && defl->R && defl->lambda, "deflation: null L, R or lambda");
    SGN_REQUIRE(defl->L != defl->R, "deflation: L and R must be different arrays");
    double lmax = 0.0;
    for (int i = 0; i < m; ++i) {
        const double re = defl->lambda[2 * i], im = defl->lambda[2 * i + 1];
        SGN_REQUIRE(std::isfinite(re) && std::isfinite(im), "deflation: eigenvalue not finite");
        lmax = std::max(lmax, std::hypot(re, im));
    }
    // scratch: c (2m: L^H b, R^H b), d (m: signs), v (m: probe), w (m: L^H R v),
    // nl (m: ||l_i||^2), nu (1: ||R v||^2)
    z64 *sc = static_cast<z64 *>(ctx.ensure_small(sizeof(z64) * (6 * (size_t)m + 1)));
    z64 *c = sc, *d = sc + 2 * m, *v = sc + 3 * m, *w = sc + 4 * m, *nl = sc + 5 * m, *nu = sc + 6 * m;
    std::vector<z64> host(2 * (size_t)m);  // signs, then the probe
    for (int i = 0; i < m; ++i) {
        const double re = defl->lambda[2 * i];
        if (!(std::abs(re) > 1e-12 * lmax)) throw Failure{SGN_ERR_IMAG_AXIS, "deflated eigenvalue on the imaginary axis"};
        host[i] = {re > 0 ? 1.0 : -1.0, 0.0};
        host[m + i] = {std::cos(0.7 + 1.3 * i), std::sin(0.7 + 1.3 * i)};
    }
    check = check && r != nullptr;
    if (x || check) SGN_HIP(hipMemcpyAsync(d, host.data(), sizeof(z64) * 2 * m, hipMemcpyHostToDevice, s));
    if (check) {
        // L^H R = I (the oblique projector P = R L^H of the deflation section): probe it with v
        deflate_combine(r, {0.0, 0.0}, {1.0, 0.0}, defl->R, m, v, nullptr, n, s);  // u = R v
        deflate_dots(defl->L, m, r, n, w, ctx, s);                                 // L^H u
        deflate_norms(defl->L, m, n, nl, ctx, s);
        const int nb = norm2_partials(r, n, false, static_cast<z64 *>(ctx.ensure_partials((kMaxBlocks + 1) * sizeof(z64))), s);
        finalize_sum(static_cast<z64 *>(ctx.partials), nb, nu, s);
        std::vector<z64> got(2 * (size_t)m + 1);
        SGN_HIP(hipMemcpyAsync(got.data(), w, sizeof(z64) * (2 * m + 1), hipMemcpyDeviceToHost, s));
        SGN_HIP(hipStreamSynchronize(s));
        const double un = std::sqrt(got[2 * m].r);
        for (int i = 0; i < m; ++i) {
            const z64 e = got[i] - host[m + i];
            const double lim = kBiorthTol * std::sqrt(got[m + i].r) * un;
            if (!(std::sqrt(norm2(e)) <= lim))
                throw Failure{SGN_ERR_INVALID, "deflation: L^H R differs from the identity (row " + std::to_string(i) +
                                                   ", |(L^H R v - v)_i| = " + std::to_string(std::sqrt(norm2(e))) + ")"};
        }
    } else if (x) {
        SGN_HIP(hipStreamSynchronize(s));  // the host signs are uploaded
    }
    if (r) SGN_HIP(hipMemcpyAsync(r, b, bytes, hipMemcpyDeviceToDevice, s));
    if (rt) SGN_HIP(hipMemcpyAsync(rt, b, bytes, hipMemcpyDeviceToDevice, s));
    deflate_dots(defl->L, m, b, n, c, ctx, s);  // L^H b
    if (x) deflate_combine(x, {0.0, 0.0}, {1.0, 0.0}, defl->R, m, c, d, n, s);
    if (r) deflate_combine(r, {1.0, 0.0}, {-1.0, 0.0}, defl->R, m, c, nullptr, n, s);
    if (rt) {
        deflate_dots(defl->R, m, b, n, c + m, ctx, s);  // R^H b
        deflate_combine(rt, {1.0, 0.0}, {-1.0, 0.0}, defl->L, m, c + m, nullptr, n, s);
    }
}

namespace {
// x += c v  (second pass of the two-pass form)
__global__ void lz_accum_kernel(double2 *x, z64 c, const double2 *v, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 xv = x[e], vv = v[e];
        const z64 r = z64{xv.x, xv.y} + c * z64{vv.x, vv.y};
        x[e] = make_double2(r.r, r.i);
    }
}
}  // namespace

}  // namespace sgn

using namespace sgn;

extern "C" sgn_status sign_lanczos_2sided(sgn_lattice l, double mu, const void *b, void *x,
                                          const sgn_deflation *defl, const sgn_lanczos_opts *opts,
                                          sgn_stats *stats, void *stream)
{
    return guard([&] {
        const auto t_start = std::chrono::steady_clock::now();
        SGN_REQUIRE(l && b && x && opts, "sign_lanczos_2sided: null argument");
        SGN_REQUIRE(opts->k >= 1, "sign_lanczos_2sided: k must be >= 1");
        SGN_REQUIRE(std::isfinite(mu), "sign_lanczos_2sided: mu not finite");
        Lattice &lat = *as_lattice(l);
        Context &ctx = *lat.ctx;
        SGN_HIP(hipSetDevice(ctx.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int k = opts->k;
        // canonical vectors have n = 12 V entries, internal ones ni = 12 S (padded stride)
        const int64_t V = lat.V, Sst = lat.S, n = 12 * V, ni = 12 * Sst;
        const size_t b64 = (size_t)n * 16, i64 = (size_t)ni * 16, b32 = (size_t)ni * 8;
        const bool f32 = opts->prec != SGN_PREC_F64;
        const sgn_prec sp = opts->prec;
        if (stats) *stats = sgn_stats{};

        // canonical residual and shadow; x <- x_P
        DevBuf r(b64), rt(b64);
        deflation_prologue(ctx, defl, n, b, x, r.p, rt.p, s);
        const double beta = norm_sync(ctx, r.p, n, false, s);
        SGN_REQUIRE(std::isfinite(beta), "sign_lanczos_2sided: b contains NaN or Inf");
        // (I - P) b at rounding level: the deflated part x_P is the whole answer
        if (beta <= 1e-13 * norm_sync(ctx, b, n, false, s)) return;
        const z64 g = dot_sync(ctx, r.p, rt.p, n, false, s);   // r^H r~
        if (!(std::sqrt(norm2(g)) > 1e-14 * beta * norm_sync(ctx, rt.p, n, false, s)))
            throw Failure{SGN_ERR_BREAKDOWN, "shadow vector orthogonal to the residual"};

        // workspace: basis V (k vectors, or a ring of 3 in the two-pass form), 3 W vectors,
        // u, z (FP64 internal) + FP32 copies
        const bool two_pass = opts->two_pass != 0;
        // basis: stored vectors from the context's pool, or a ring of 3 in the two-pass form
        DevBuf ring(two_pass ? 3 * i64 : 0), Wb(3 * i64), u(i64), z(i64);
        PooledBasis basis(ctx, i64, (size_t)k, "sign_lanczos_2sided");
        if (!two_pass) basis.ensure(0);
        DevBuf v32(f32 ? b32 : 0), w32(f32 ? b32 : 0), u32(f32 ? b32 : 0), z32(f32 ? b32 : 0);
        DevBuf scal(sizeof(z64) * (5 * (size_t)k + 2) + sizeof(int) * k);
        LzScalars S;
        S.alpha = scal.as<z64>();
        S.hsub = S.alpha + k;
        S.hsup = S.hsub + k;
        S.sv = S.hsup + k;
        S.tw = S.sv + (k + 1);
        S.flag = reinterpret_cast<int *>(S.tw + (k + 1));
        const double s1 = 1.0 / beta;
        const z64 v1rt = {s1 * g.r, s1 * g.i};  // v_1^H r~
        const double m2 = norm2(v1rt);
        const z64 t1 = {v1rt.r / m2, -v1rt.i / m2};  // 1 / (v_1^H r~)
        const z64 sv0 = {s1, 0.0};
        auto Vj = [&](int j) {
            return two_pass ? static_cast<char *>(ring.p) + (size_t)(j % 3) * i64 : static_cast<char *>(basis[j]);
        };
        auto Wj = [&](int j) { return static_cast<char *>(Wb.p) + (size_t)(j % 3) * i64; };
        // start of the recurrence (run once, or twice in the two-pass form, from identical state)
        auto start = [&]() {
            SGN_HIP(hipMemsetAsync(scal.p, 0, sizeof(z64) * (5 * (size_t)k + 2) + sizeof(int) * k, s));
            SGN_HIP(hipMemcpyAsync(S.sv, &sv0, sizeof(z64), hipMemcpyHostToDevice, s));
            SGN_HIP(hipMemcpyAsync(S.tw, &t1, sizeof(z64), hipMemcpyHostToDevice, s));
            pack_spinor(lat, r.p, Vj(0), SGN_PREC_F64, s);
            pack_spinor(lat, rt.p, Wj(0), SGN_PREC_F64, s);
            if (f32) {
                convert_64_to_32(Vj(0), v32.p, Sst, s);
                convert_64_to_32(Wj(0), w32.p, Sst, s);
            }
        };
        start();

        const int nst = dslash_blocks(lat);
        const int nvb = vec_blocks(6 * Sst);
        z64 *part = static_cast<z64 *>(ctx.ensure_partials(sizeof(z64) * std::max(nst, 2 * nvb)));
        OpSpec opA, opAh;
        opA.mu = mu;
        opAh.mu = -mu;

        std::vector<z64> halpha(k), hsub(k), hsup(k), hsv(k + 1), ycur, yprev;
        std::vector<int> hflag(k);
        auto download = [&](int kk) {
            SGN_HIP(hipMemcpyAsync(halpha.data(), S.alpha, sizeof(z64) * kk, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipMemcpyAsync(hsub.data(), S.hsub, sizeof(z64) * kk, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipMemcpyAsync(hsup.data(), S.hsup, sizeof(z64) * kk, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipMemcpyAsync(hsv.data(), S.sv, sizeof(z64) * kk, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipMemcpyAsync(hflag.data(), S.flag, sizeof(int) * kk, hipMemcpyDeviceToHost, s));
            SGN_HIP(hipStreamSynchronize(s));
            for (int j = 0; j + 1 < kk; ++j)
                if (hflag[j]) throw Failure{SGN_ERR_BREAKDOWN, "two-sided Lanczos breakdown at step " + std::to_string(j + 1)};
        };
        double small_ms = 0.0, minre = 0.0;
        auto small_sign = [&](int kk, std::vector<z64> &y) {
            const auto t0 = std::chrono::steady_clock::now();
            std::vector<std::complex<double>> d(kk), sb(kk), sp(kk), yy(kk);
            for (int j = 0; j < kk; ++j) {
                d[j] = {halpha[j].r, halpha[j].i};
                sb[j] = {hsub[j].r, hsub[j].i};
                sp[j] = {hsup[j].r, hsup[j].i};
            }
            SmallSignInfo info;
            const int rc = small_sign_e1(kk, d.data(), sb.data(), sp.data(), yy.data(), &info);
            small_ms += ms_since(t0);
            minre = info.min_abs_re;
            if (rc == 3) throw Failure{SGN_ERR_IMAG_AXIS, "eigenvalue of T_k on the imaginary axis"};
            if (rc != 0) throw Failure{SGN_ERR_INVALID, "small sign: QR iteration failed"};
            y.resize(kk);
            for (int j = 0; j < kk; ++j) y[j] = {yy[j].real(), yy[j].imag()};
        };

        // one step j of the recurrence: alpha_j, and (unless last) v_{j+1}, w_{j+1}
        auto step = [&](int j, int last) {
            // u = A vh_j with partials of wh_j^H u
            Epilogue ep;
            ep.w = f32 ? w32.p : Wj(j);
            ep.partials = part;
            const int nb1 = dslash_launch(lat, sp, opA, f32 ? v32.p : Vj(j), f32 ? u32.p : u.p, ep, s);
            hipLaunchKernelGGL(lz_alpha_kernel, dim3(1), dim3(256), 0, s, part, nb1, S, j);
            if (j + 1 == last) return;
            if (!two_pass) basis.ensure(j + 1);
            dslash_launch(lat, sp, opAh, f32 ? w32.p : Wj(j), f32 ? z32.p : z.p, Epilogue{}, s);
            void *vn = Vj(j + 1);
            const double2 *vjm = j > 0 ? reinterpret_cast<const double2 *>(Vj(j - 1)) : nullptr;
            const double2 *wjm = j > 0 ? reinterpret_cast<const double2 *>(Wj(j - 1)) : nullptr;
            if (f32)
                hipLaunchKernelGGL(lz_update_kernel<true>, dim3(nvb), dim3(256), 0, s, u32.p, z32.p,
                                   (const double2 *)Vj(j), vjm, (const double2 *)Wj(j), wjm, (double2 *)vn,
                                   (double2 *)Wj(j + 1), (float4 *)v32.p, (float4 *)w32.p, (double2 *)nullptr,
                                   (double2 *)nullptr, S, j, (int)Sst, part);
            else
                hipLaunchKernelGGL(lz_update_kernel<false>, dim3(nvb), dim3(256), 0, s, u.p, z.p,
                                   (const double2 *)Vj(j), vjm, (const double2 *)Wj(j), wjm, (double2 *)vn,
                                   (double2 *)Wj(j + 1), (float4 *)nullptr, (float4 *)nullptr, (double2 *)nullptr,
                                   (double2 *)nullptr, S, j, (int)Sst, part);
            hipLaunchKernelGGL(lz_step_kernel, dim3(1), dim3(256), 0, s, part, nvb, S, j, 1e-14);
            SGN_HIP(hipGetLastError());
        };

        const auto t_kry = std::chrono::steady_clock::now();
        int kused = k, checked = 0;  // checked: size of the last small sign computed in the loop
        // With an early stop, T_kk is downloaded at every check point kk and the next check_every
        // steps are queued before the host evaluates sign(T_kk) e_1, so the host's small sign and the
        // device's Lanczos steps overlap.  When the check stops at kk, the steps queued beyond it are
        // discarded (they do not change steps < kk: the same launches give the same results).
        const bool adaptive = opts->tol > 0 && opts->check_every > 0;
        const int ce = adaptive ? opts->check_every : k;
        int launched = 0;
        auto launch_to = [&](int upto) {
            for (; launched < upto; ++launched) step(launched, k);
        };
        launch_to(std::min(ce, k));
        while (adaptive && launched < k) {
            const int kk = launched;
            download(kk);
            launch_to(std::min(kk + ce, k));
            small_sign(kk, ycur);
            checked = kk;
            if (!yprev.empty()) {
                double num = 0.0, den = 0.0;
                for (int i = 0; i < kk; ++i) {
                    z64 d = ycur[i];
                    if (i < (int)yprev.size()) d = d - yprev[i];
                    num += norm2(d);
                    den += norm2(ycur[i]);
                }
                if (std::sqrt(num) <= opts->tol * std::sqrt(den)) {
                    kused = kk;
                    break;
                }
            }
            yprev = ycur;
        }
        SGN_HIP(hipGetLastError());
        download(kused);
        const double kry_ms = ms_since(t_kry);
        std::vector<z64> y;
        if (checked == kused)
            y = ycur;  // the stopping check already computed sign(T_k) e_1 for this k
        else
            small_sign(kused, y);
        // x = x_P + beta * sum_j y_j s_j vh_j
        std::vector<z64> c(kused);
        for (int j = 0; j < kused; ++j) c[j] = (beta * hsv[j].r) * y[j];
        DevBuf cd(sizeof(z64) * kused), tab(sizeof(void *) * kused);
        if (!two_pass) {
            SGN_HIP(hipMemcpyAsync(cd.p, c.data(), sizeof(z64) * kused, hipMemcpyHostToDevice, s));
            SGN_HIP(hipMemcpyAsync(tab.p, basis.slots.data(), sizeof(void *) * kused, hipMemcpyHostToDevice, s));
            basis.lift(cd.as<z64>(), static_cast<const void *const *>(tab.p), kused, ni, u.p, s);
        } else {
            // second pass: the same launches from the same state give the same vh_j bit for bit;
            // each is added to the solution while it is still in the ring.  x accumulates in xacc
            // (the first pass is done with the canonical shadow rt, reused here)
            DevBuf xacc(i64);
            SGN_HIP(hipMemsetAsync(xacc.p, 0, i64, s));
            start();
            for (int j = 0; j < kused; ++j) {
                hipLaunchKernelGGL(lz_accum_kernel, dim3(vec_blocks(ni)), dim3(256), 0, s, (double2 *)xacc.p, c[j],
                                   (const double2 *)Vj(j), ni);
                if (j + 1 < kused) step(j, kused);
            }
            SGN_HIP(hipMemcpyAsync(u.p, xacc.p, i64, hipMemcpyDeviceToDevice, s));
        }
        unpack_spinor(lat, u.p, r.p, SGN_PREC_F64, s);
        axpby64({1.0, 0.0}, r.p, {1.0, 0.0}, x, n, s);
        SGN_HIP(hipStreamSynchronize(s));
        if (stats) {
            stats->iterations = kused;
            stats->matvecs = 2 * launched - (launched == k ? 1 : 0) + (two_pass ? 2 * (kused - 1) : 0);
            stats->min_abs_re = minre;
            stats->krylov_ms = kry_ms;
            stats->small_ms = small_ms;
            stats->total_ms = ms_since(t_start);
        }
    });
}

// ---------------------------------------------------------------------------
// Multishift QMR (the QMR variant named beside BiCG in the section "Two-sided
// Lanczos with rational functions"; shifted QMR after Freund).
//
// One two-sided Lanczos sequence on A' = c^2 H_W(mu)^2 (the recurrence above,
// each operator application two stencils with the c^2 folded into the second
// one's epilogue), v_1 = y/||y||, shadow w_1 = v_1, y = c H_W (I - P) b.
// Shift invariance: (A' - sigma_i) V_k = V_{k+1} (Tbar_k - sigma_i Ibar_k), so
// the QMR iterate of every shift is x_i = V_k z_i with z_i the least-squares
// solution of min || ||y|| e_1 - (Tbar_k - sigma_i Ibar_k) z ||.  The host
// keeps a Givens QR of each shifted tridiagonal, one column per step, whose
// last rotated right-hand side entry is the quasi-residual tau_i.  Every
// basis vector vh_j is stored (one pooled slot per step); the result
// sum_i omega_i x_i = V_k (sum_i omega_i z_i) is one lift at the end.
namespace sgn {
namespace {

using cplx = std::complex<double>;

// Givens QR of the shifted (k+1) x k tridiagonal Tbar_k - sigma Ibar_k, built
// one column per Lanczos step.  R is upper triangular with two superdiagonals.
struct QmrShift {
    double sigma = 0.0;
    std::vector<cplx> rd, r1, r2;  // R_jj, R_{j-1,j}, R_{j-2,j} of column j
    std::vector<double> gc;        // rotation j acts on rows (j, j+1): [c s; -conj(s) c]
    std::vector<cplx> gs;
    std::vector<cplx> g;           // rotated right-hand side, k+1 entries
    static void rot(double c, cplx s, cplx &a, cplx &b)
    {
        const cplx t = c * a + s * b;
        b = -std::conj(s) * a + c * b;
        a = t;
    }
    // column j: h_{j-1,j} (zero for j = 0), h_jj - sigma, h_{j+1,j}
    bool add_column(int j, cplx hsup_prev, cplx alpha, double hsub)
    {
        cplx x0 = 0.0, x1 = j >= 1 ? hsup_prev : cplx(0.0), x2 = alpha - sigma, x3 = hsub;
        if (j >= 2) rot(gc[j - 2], gs[j - 2], x0, x1);
        if (j >= 1) rot(gc[j - 1], gs[j - 1], x1, x2);
        const double a = std::abs(x2), b = std::abs(x3), r = std::hypot(a, b);
        if (!(r > 0.0)) return false;
        const double c = a / r;
        const cplx s = a > 0.0 ? (x2 / a) * std::conj(x3) / r : std::conj(x3) / b;
        rd.push_back(c * x2 + s * x3);
        r1.push_back(x1);
        r2.push_back(x0);
        gc.push_back(c);
        gs.push_back(s);
        const cplx gj = g[j];
        g[j] = c * gj;
        g.push_back(-std::conj(s) * gj);
        return true;
    }
    double tau() const { return std::abs(g.back()); }
    // z of the first k columns (back substitution)
    std::vector<cplx> solve(int k) const
    {
        std::vector<cplx> z(k);
        for (int j = k - 1; j >= 0; --j) {
            cplx t = g[j];
            if (j + 1 < k) t -= r1[j + 1] * z[j + 1];
            if (j + 2 < k) t -= r2[j + 2] * z[j + 2];
            z[j] = t / rd[j];
        }
        return z;
    }
};

// One problem of multishift QMR: setup, the Lanczos steps (launched one by one for a single problem,
// or by QmrBatch for several in lockstep), the host's absorption of finished steps (a Givens column
// per shift), the precision schedule, and the final lift.
class QmrSolve {
  public:
    // pool_next (a batch): the next unused buffer of each per-size pool, shared by the batch's problems
    QmrSolve(const sgn_problem &pb, const sgn_rational &rf, const sgn_ms_opts &o, hipStream_t s,
             std::map<size_t, size_t> *pool_next = nullptr)
        : pb_(pb), rf_(rf), o_(o), s_(s), lat_(*as_lattice(pb.lat)), ctx_(*lat_.ctx), pool_next_(pool_next)
    {
    }
    // x = x_P, y = c H (I - P) b; false if y = 0 (x = x_P is written, nothing else to do)
    bool setup(sgn_stats *st, bool batch);
    void step(int j);  // one Lanczos step on A' (single-problem form)
    // the steps j0 .. launched-1 have run: their coefficients into every shift's QR; true once done
    bool absorb(int j0, int launched);
    bool absorb_host(int j0, int launched);  // absorb with the coefficients copied in already
    bool switch_precision();  // the mixed schedule after a chunk; true if the phase changed
    sgn_status finish(sgn_stats *st);
    sgn_status run(sgn_stats *st);

  private:
    friend class QmrBatch;
    const sgn_problem &pb_;
    const sgn_rational &rf_;
    const sgn_ms_opts &o_;
    hipStream_t s_;
    Lattice &lat_;
    Context &ctx_;
    std::map<size_t, size_t> *pool_next_;
    int64_t V_ = 0, Sst_ = 0, nc_ = 0, ni_ = 0;
    size_t b64_ = 0, i64_ = 0, b32_ = 0;
    bool mixed_ = false, f32_ = false;
    double theta32_ = 0.0, theta16_ = 0.0, c2_ = 0.0, ynorm_ = 0.0, small_ms_ = 0.0;
    sgn_prec sp_ = SGN_PREC_F64;
    int ns_ = 0, maxiter_ = 0, poll_ = 4, nst_ = 0, nvb_ = 0;
    OpSpec opA_, opAh_;
    std::unique_ptr<DevBuf> rcan_, y_, tmp_, Wb_, u_, z_, v32_, w32_, t32_, u32_, z32_, scal_;
    std::unique_ptr<PooledBasis> basis_;
    LzScalars S_{};
    z64 *part_ = nullptr;
    std::vector<QmrShift> G_;
    std::vector<z64> halpha_, hsub_, hsup_;
    std::vector<int> hflag_;
    sgn_status result_ = SGN_OK;
    int launched_ = 0, kused_ = -1;
    std::chrono::steady_clock::time_point t_start_, t_kry_;
    // batch form: stencil inputs at fixed addresses, a device step counter and done flag, own partials
    std::unique_ptr<DevBuf> vcur_, wcur_, bpart_, dslot_buf_;
    void **dslots_ = nullptr;  // device copy of the basis slot table (batch form)
    size_t dslots_n_ = 0;
    int *dstep_ = nullptr, *ddone_ = nullptr;
    z64 *part1_ = nullptr, *part2_ = nullptr;
    void ensure_slots(int upto);  // slots 0 .. upto, and their device table

    char *Wj(int j) const { return static_cast<char *>(Wb_->p) + (size_t)(j % 3) * i64_; }
};

bool QmrSolve::setup(sgn_stats *st, bool batch)
{
    t_start_ = std::chrono::steady_clock::now();
    SGN_HIP(hipSetDevice(ctx_.device));
    V_ = lat_.V;
    Sst_ = lat_.S;
    nc_ = 12 * V_;
    ni_ = 12 * Sst_;
    b64_ = (size_t)nc_ * 16;
    i64_ = (size_t)ni_ * 16;
    b32_ = (size_t)ni_ * 8;
    // precision schedule: FP64 steps while the largest quasi-residual is above theta32 ||y||,
    // then the stencil in FP32 (and with FP16 links below theta16 ||y|| for SGN_PREC_F32_H16);
    // the recurrences and the basis stay FP64
    mixed_ = o_.prec != SGN_PREC_F64;
    theta32_ = mixed_ ? (o_.theta32 > 0 ? o_.theta32 : 1e-3) : 0.0;
    theta16_ = o_.prec == SGN_PREC_F32_H16 ? (o_.theta16 > 0 ? o_.theta16 : 1e-6) : 0.0;
    ns_ = rf_.s;
    c2_ = rf_.c * rf_.c;
    maxiter_ = o_.maxiter > 0 ? o_.maxiter : 10000;
    poll_ = o_.poll > 0 ? o_.poll : 4;
    if (st) {
        *st = sgn_stats{};
        st->nshift = ns_;
    }
    opA_.mu = pb_.mu;
    opAh_.mu = -pb_.mu;

    // x <- x_P, y = c H (I - P) b
    rcan_ = std::make_unique<DevBuf>(b64_);
    y_ = std::make_unique<DevBuf>(i64_);
    tmp_ = std::make_unique<DevBuf>(i64_);
    deflation_prologue(ctx_, pb_.defl, nc_, pb_.b, pb_.x, rcan_->p, nullptr, s_);
    pack_spinor(lat_, rcan_->p, tmp_->p, SGN_PREC_F64, s_);
    {
        Epilogue ep;
        ep.a = rf_.c;
        dslash_launch(lat_, SGN_PREC_F64, opA_, tmp_->p, y_->p, ep, s_);
    }
    ynorm_ = norm_sync(ctx_, y_->p, ni_, false, s_);
    SGN_REQUIRE(std::isfinite(ynorm_), "multishift_qmr: b contains NaN or Inf");
    if (ynorm_ == 0.0) {  // x = x_P
        if (pb_.x_shift)
            for (int i = 0; i < ns_; ++i)
                if (pb_.x_shift[i]) SGN_HIP(hipMemsetAsync(pb_.x_shift[i], 0, b64_, s_));
        SGN_HIP(hipStreamSynchronize(s_));
        return false;
    }

    // stored basis: slot j holds vh_j (FP64, internal layout), from the context's pool
    size_t cap;
    if (o_.basis_slots > 0) {
        cap = (size_t)o_.basis_slots;
    } else {
        size_t fr = 0, tot = 0;
        SGN_HIP(hipMemGetInfo(&fr, &tot));
        cap = ctx_.basis_pools[i64_].size() + fr / 2 / i64_;
    }
    basis_ = std::make_unique<PooledBasis>(ctx_, i64_, cap, "multishift_qmr");
    if (pool_next_) basis_->shared_next = &(*pool_next_)[i64_];
    basis_->ensure(0);
    Wb_ = std::make_unique<DevBuf>(3 * i64_);
    u_ = std::make_unique<DevBuf>(i64_);
    z_ = std::make_unique<DevBuf>(i64_);
    const size_t f = mixed_ ? b32_ : 0;
    v32_ = std::make_unique<DevBuf>(f);
    w32_ = std::make_unique<DevBuf>(f);
    t32_ = std::make_unique<DevBuf>(f);
    u32_ = std::make_unique<DevBuf>(f);
    z32_ = std::make_unique<DevBuf>(f);
    const size_t nscal = sizeof(z64) * (5 * (size_t)maxiter_ + 2) + sizeof(int) * (maxiter_ + 2);
    scal_ = std::make_unique<DevBuf>(nscal);
    S_.alpha = scal_->as<z64>();
    S_.hsub = S_.alpha + maxiter_;
    S_.hsup = S_.hsub + maxiter_;
    S_.sv = S_.hsup + maxiter_;
    S_.tw = S_.sv + (maxiter_ + 1);
    S_.flag = reinterpret_cast<int *>(S_.tw + (maxiter_ + 1));
    const z64 s0 = {1.0 / ynorm_, 0.0};  // v_1 = s_0 y,  w_1 = t_0 y = v_1
    SGN_HIP(hipMemsetAsync(scal_->p, 0, nscal, s_));
    SGN_HIP(hipMemcpyAsync(S_.sv, &s0, sizeof(z64), hipMemcpyHostToDevice, s_));
    SGN_HIP(hipMemcpyAsync(S_.tw, &s0, sizeof(z64), hipMemcpyHostToDevice, s_));
    SGN_HIP(hipMemcpyAsync((*basis_)[0], y_->p, i64_, hipMemcpyDeviceToDevice, s_));
    SGN_HIP(hipMemcpyAsync(Wj(0), y_->p, i64_, hipMemcpyDeviceToDevice, s_));
    nst_ = dslash_blocks(lat_);
    nvb_ = vec_blocks(6 * Sst_);
    if (batch) {
        // the step counter and done flag live after the flags; own partials (the context's are shared)
        dstep_ = S_.flag + maxiter_;
        ddone_ = dstep_ + 1;
        vcur_ = std::make_unique<DevBuf>(i64_);
        wcur_ = std::make_unique<DevBuf>(i64_);
        SGN_HIP(hipMemcpyAsync(vcur_->p, y_->p, i64_, hipMemcpyDeviceToDevice, s_));
        SGN_HIP(hipMemcpyAsync(wcur_->p, y_->p, i64_, hipMemcpyDeviceToDevice, s_));
        const size_t n1 = (size_t)nst_, n2 = 2 * (size_t)kMaxBlocks;
        bpart_ = std::make_unique<DevBuf>(sizeof(z64) * (n1 + n2));
        part1_ = bpart_->as<z64>();
        part2_ = part1_ + n1;
        dslot_buf_ = std::make_unique<DevBuf>(sizeof(void *) * ((size_t)maxiter_ + poll_ + 2));
        dslots_ = dslot_buf_->as<void *>();
        ensure_slots(0);
    } else {
        part_ = static_cast<z64 *>(ctx_.ensure_partials(sizeof(z64) * std::max(nst_, 2 * nvb_)));
    }
    G_.assign(ns_, QmrShift{});
    for (int i = 0; i < ns_; ++i) {
        G_[i].sigma = rf_.sigma[i];
        G_[i].g.assign(1, cplx(ynorm_, 0.0));
    }
    halpha_.assign(maxiter_, {});
    hsub_.assign(maxiter_, {});
    hsup_.assign(maxiter_, {});
    hflag_.assign(maxiter_, 0);
    SGN_HIP(hipStreamSynchronize(s_));
    t_kry_ = std::chrono::steady_clock::now();
    return true;
}

// one Lanczos step on A': alpha_j, vh_{j+1}, wh_{j+1}, h_{j+1,j}, h_{j,j+1}
void QmrSolve::step(int j)
{
    const bool f32 = f32_;
    PooledBasis &basis = *basis_;
    char *tmp = static_cast<char *>(tmp_->p), *u = static_cast<char *>(u_->p), *z = static_cast<char *>(z_->p);
    dslash_launch(lat_, sp_, opA_, f32 ? v32_->p : basis[j], f32 ? t32_->p : tmp, Epilogue{}, s_);
    Epilogue ep;  // u = c^2 H (H vh_j), partials of wh_j^H u
    ep.a = c2_;
    ep.w = f32 ? w32_->p : Wj(j);
    ep.partials = part_;
    const int nb1 = dslash_launch(lat_, sp_, opA_, f32 ? t32_->p : tmp, f32 ? u32_->p : u, ep, s_);
    hipLaunchKernelGGL(lz_alpha_kernel, dim3(1), dim3(256), 0, s_, part_, nb1, S_, j);
    dslash_launch(lat_, sp_, opAh_, f32 ? w32_->p : Wj(j), f32 ? t32_->p : tmp, Epilogue{}, s_);
    Epilogue ez;  // z = c^2 H^H (H^H wh_j)
    ez.a = c2_;
    dslash_launch(lat_, sp_, opAh_, f32 ? t32_->p : tmp, f32 ? z32_->p : z, ez, s_);
    const double2 *vjm = j > 0 ? static_cast<const double2 *>(basis[j - 1]) : nullptr;
    const double2 *wjm = j > 0 ? reinterpret_cast<const double2 *>(Wj(j - 1)) : nullptr;
    const int pr = ctx_.prof_start(s_, SGN_K_SEED_UPDATE, true);
    if (f32)
        launch_k(ctx_.prof_stamp(pr), lz_update_kernel<true>, dim3(nvb_), dim3(256), 0u, s_, u32_->p, z32_->p,
                           (const double2 *)basis[j], vjm, (const double2 *)Wj(j), wjm, (double2 *)basis[j + 1],
                           (double2 *)Wj(j + 1), (float4 *)v32_->p, (float4 *)w32_->p, (double2 *)nullptr,
                           (double2 *)nullptr, S_, j, (int)Sst_, part_);
    else
        launch_k(ctx_.prof_stamp(pr), lz_update_kernel<false>, dim3(nvb_), dim3(256), 0u, s_, u, z, (const double2 *)basis[j],
                           vjm, (const double2 *)Wj(j), wjm, (double2 *)basis[j + 1], (double2 *)Wj(j + 1),
                           (float4 *)nullptr, (float4 *)nullptr, (double2 *)nullptr, (double2 *)nullptr, S_, j,
                           (int)Sst_, part_);
    const double io = (f32 ? 2.0 * b32_ : 2.0 * i64_) + (j > 0 ? 4.0 : 2.0) * i64_ + 2.0 * i64_ + (f32 ? 2.0 * b32_ : 0.0);
    ctx_.prof_stop(pr, s_, SGN_K_SEED_UPDATE, io, 40.0 * ni_);
    hipLaunchKernelGGL(lz_step_kernel, dim3(1), dim3(256), 0, s_, part_, nvb_, S_, j, 1e-14);
    SGN_HIP(hipGetLastError());
}

void QmrSolve::ensure_slots(int upto)
{
    basis_->ensure(upto);
    const size_t n = basis_->slots.size();
    if (dslots_ && n > dslots_n_) {
        SGN_HIP(hipMemcpy(dslots_ + dslots_n_, basis_->slots.data() + dslots_n_, sizeof(void *) * (n - dslots_n_),
                          hipMemcpyHostToDevice));
        dslots_n_ = n;
    }
}

bool QmrSolve::absorb(int j0, int launched)
{
    const int nn = launched - j0;
    SGN_HIP(hipMemcpyAsync(halpha_.data() + j0, S_.alpha + j0, sizeof(z64) * nn, hipMemcpyDeviceToHost, s_));
    SGN_HIP(hipMemcpyAsync(hsub_.data() + j0, S_.hsub + j0, sizeof(z64) * nn, hipMemcpyDeviceToHost, s_));
    SGN_HIP(hipMemcpyAsync(hsup_.data() + j0, S_.hsup + j0, sizeof(z64) * nn, hipMemcpyDeviceToHost, s_));
    SGN_HIP(hipMemcpyAsync(hflag_.data() + j0, S_.flag + j0, sizeof(int) * nn, hipMemcpyDeviceToHost, s_));
    SGN_HIP(hipStreamSynchronize(s_));
    return absorb_host(j0, launched);
}

// the coefficients of steps j0 .. launched-1 are on the host already
bool QmrSolve::absorb_host(int j0, int launched)
{
    const auto t0 = std::chrono::steady_clock::now();
    for (int j = j0; j < launched; ++j) {
        const cplx al(halpha_[j].r, halpha_[j].i), hp = j > 0 ? cplx(hsup_[j - 1].r, hsup_[j - 1].i) : cplx(0.0);
        double tmax = 0.0;
        for (auto &g : G_) {
            if (!g.add_column(j, hp, al, hsub_[j].r))
                throw Failure{SGN_ERR_BREAKDOWN, "multishift_qmr: singular shifted tridiagonal"};
            tmax = std::max(tmax, g.tau());
        }
        if (!std::isfinite(tmax)) throw Failure{SGN_ERR_BREAKDOWN, "multishift_qmr: non-finite Lanczos coefficients"};
        if (tmax <= o_.tol * ynorm_ || hsub_[j].r == 0.0) {  // converged, or invariant subspace (exact)
            kused_ = j + 1;
            break;
        }
        if (hflag_[j]) throw Failure{SGN_ERR_BREAKDOWN, "two-sided Lanczos breakdown at step " + std::to_string(j + 1)};
    }
    small_ms_ += ms_since(t0);
    launched_ = launched;
    if (kused_ < 0 && launched >= maxiter_) {
        kused_ = launched;
        result_ = SGN_ERR_NOT_CONVERGED;
    }
    return kused_ >= 0;
}

bool QmrSolve::switch_precision()
{
    if (kused_ >= 0 || !mixed_) return false;
    double tmax = 0.0;
    for (const auto &g : G_) tmax = std::max(tmax, g.tau());
    bool changed = false;
    if (!f32_ && tmax < theta32_ * ynorm_) {  // FP32 copies of the current vh_j, wh_j
        const void *vc = vcur_ ? vcur_->p : (*basis_)[launched_];
        const void *wc = wcur_ ? wcur_->p : Wj(launched_);
        convert_64_to_32(vc, v32_->p, Sst_, s_);
        convert_64_to_32(wc, w32_->p, Sst_, s_);
        f32_ = true;
        sp_ = SGN_PREC_F32;
        changed = true;
    }
    if (f32_ && sp_ == SGN_PREC_F32 && tmax < theta16_ * ynorm_) {
        sp_ = SGN_PREC_F32_H16;
        changed = true;
    }
    return changed;
}

sgn_status QmrSolve::run(sgn_stats *st)
{
    if (!setup(st, false)) return SGN_OK;
    while (kused_ < 0) {
        const int chunk = std::min(poll_, maxiter_ - launched_);
        basis_->ensure(launched_ + chunk);
        for (int q = 0; q < chunk; ++q) step(launched_ + q);
        if (!absorb(launched_, launched_ + chunk)) switch_precision();
    }
    return finish(st);
}

sgn_status QmrSolve::finish(sgn_stats *st)
{
    const double kry_ms = ms_since(t_kry_);
    const int kused = kused_;
    const int ns = ns_;
    const hipStream_t s = s_;
    Lattice &lat = lat_;
    Context &ctx = ctx_;
    PooledBasis &basis = *basis_;
    // coefficients of the stored vectors: x_i = sum_j z_ij s_j vh_j
    std::vector<z64> hsv(kused);
    SGN_HIP(hipMemcpy(hsv.data(), S_.sv, sizeof(z64) * kused, hipMemcpyDeviceToHost));
    std::vector<std::vector<cplx>> Z(ns);
    for (int i = 0; i < ns; ++i) Z[i] = G_[i].solve(kused);
    // coefficient sets: 0 = sum_i omega_i x_i, then one per shift whose x_i is requested or
    // verified; all are uploaded before the first lift is queued (no buffer is reused)
    std::vector<int> sel;
    for (int i = 0; i < ns; ++i)
        if ((pb_.x_shift && pb_.x_shift[i]) || o_.verify) sel.push_back(i);
    const size_t nset = 1 + sel.size();
    std::vector<z64> hcoef(nset * kused);
    for (int j = 0; j < kused; ++j) {
        cplx d = 0.0;
        for (int i = 0; i < ns; ++i) d += rf_.omega[i] * Z[i][j];
        d *= hsv[j].r;
        hcoef[j] = {d.real(), d.imag()};
    }
    for (size_t q = 0; q < sel.size(); ++q)
        for (int j = 0; j < kused; ++j) {
            const cplx d = Z[sel[q]][j] * hsv[j].r;
            hcoef[(q + 1) * kused + j] = {d.real(), d.imag()};
        }
    DevBuf dtab(sizeof(void *) * kused), dcoef(sizeof(z64) * hcoef.size());
    SGN_HIP(hipMemcpy(dtab.p, basis.slots.data(), sizeof(void *) * kused, hipMemcpyHostToDevice));
    SGN_HIP(hipMemcpy(dcoef.p, hcoef.data(), sizeof(z64) * hcoef.size(), hipMemcpyHostToDevice));
    auto lift = [&](size_t set, void *out) {
        const int pr = ctx.prof_start(s, SGN_K_LIFT);
        basis.lift(dcoef.as<z64>() + set * kused, static_cast<const void *const *>(dtab.p), kused, ni_, out, s);
        ctx.prof_stop(pr, s, SGN_K_LIFT, (double)i64_ * (kused + 1), 8.0 * ni_ * kused);
    };
    // canonical v <- (I - P) v (rounding components along the deflated eigenvectors)
    const bool deflated = pb_.defl && pb_.defl->m > 0;
    DevBuf dfc(deflated ? sizeof(z64) * pb_.defl->m : 0);
    auto project_out = [&](void *v) {
        if (!deflated) return;
        deflate_dots(pb_.defl->L, pb_.defl->m, v, nc_, dfc.as<z64>(), ctx, s);
        deflate_combine(v, {1.0, 0.0}, {-1.0, 0.0}, pb_.defl->R, pb_.defl->m, dfc.as<z64>(), nullptr, nc_, s);
    };
    lift(0, tmp_->p);
    unpack_spinor(lat, tmp_->p, rcan_->p, SGN_PREC_F64, s);
    project_out(rcan_->p);
    axpby64({1.0, 0.0}, rcan_->p, {1.0, 0.0}, pb_.x, nc_, s);

    // per-shift solutions: requested ones, and all of them for the FP64 residual check
    std::vector<double> res(ns);
    for (int i = 0; i < ns; ++i) res[i] = G_[i].tau() / ynorm_;
    int extra_mv = 0;
    DevBuf h(o_.verify ? i64_ : 0), q(o_.verify ? i64_ : 0);
    for (size_t k = 0; k < sel.size(); ++k) {
        const int i = sel[k];
        lift(k + 1, tmp_->p);
        if (o_.verify) {  // r_i = y - (c^2 H^2 - sigma_i) x_i in FP64
            dslash_launch(lat, SGN_PREC_F64, opA_, tmp_->p, h.p, Epilogue{}, s);
            Epilogue ep;
            ep.a = -c2_;
            ep.z = tmp_->p;
            ep.b = {rf_.sigma[i], 0.0};
            dslash_launch(lat, SGN_PREC_F64, opA_, h.p, q.p, ep, s);
            axpby64({1.0, 0.0}, y_->p, {1.0, 0.0}, q.p, ni_, s);
            res[i] = norm_sync(ctx, q.p, ni_, false, s) / ynorm_;
            extra_mv += 2;
        }
        if (pb_.x_shift && pb_.x_shift[i]) {
            unpack_spinor(lat, tmp_->p, pb_.x_shift[i], SGN_PREC_F64, s);
            project_out(pb_.x_shift[i]);
        }
    }
    SGN_HIP(hipStreamSynchronize(s));
    if (st) {
        st->iterations = kused;
        st->matvecs = 4 * launched_ + 1 + extra_mv;
        double mx = 0.0;
        for (int i = 0; i < ns; ++i) {
            st->shift_residual[i] = res[i];
            mx = std::max(mx, res[i]);
        }
        st->residual = mx;
        st->krylov_ms = kry_ms;
        st->small_ms = small_ms_;
        st->total_ms = ms_since(t_start_);
    }
    return result_;
}

// Lockstep batch of QMR problems: one descriptor per problem in device memory; the step index comes
// from the problem's device counter (advanced by its step kernel), so a chunk of steps is one graph
// replayed until a problem changes precision or several have finished.  The stencils read the
// current basis vectors from fixed copies (vcur, wcur in FP64; the FP32 copies in the FP32 phases).
struct QbDesc {
    LzScalars S;
    int *step, *done;
    void *const *slots;  // basis slot table
    double2 *W[3];       // the W ring
    double2 *vcur, *wcur;
    float4 *v32, *w32;
    const void *u, *z;   // stencil outputs of the problem's phase
    z64 *part1, *part2;
    int nb1, Sst;
};

__global__ void __launch_bounds__(256) qb_alpha_batch(const QbDesc *d)
{
    const QbDesc &D = d[blockIdx.x];
    if (*D.done) return;
    lz_alpha_body(D.part1, D.nb1, D.S, *D.step);
}

template <bool F32>
__global__ void __launch_bounds__(256) qb_update_batch(const QbDesc *d)
{
    const QbDesc &D = d[blockIdx.y];
    if (*D.done) return;
    const int j = *D.step;
    const double2 *vj = static_cast<const double2 *>(D.slots[j]);
    const double2 *vjm = j > 0 ? static_cast<const double2 *>(D.slots[j - 1]) : nullptr;
    lz_update_body<F32>(D.u, D.z, vj, vjm, D.W[j % 3], j > 0 ? D.W[(j + 2) % 3] : nullptr,
                        static_cast<double2 *>(D.slots[j + 1]), D.W[(j + 1) % 3], D.v32, D.w32,
                        F32 ? nullptr : D.vcur, F32 ? nullptr : D.wcur, D.S, j, D.Sst, D.part2);
}

// nb: the grid width of the update that wrote the partials
__global__ void __launch_bounds__(256) qb_step_batch(const QbDesc *d, int nb)
{
    const QbDesc &D = d[blockIdx.x];
    if (*D.done) return;
    const int j = *D.step;
    lz_step_body(D.part2, nb, D.S, j, 1e-14);
    if (threadIdx.x == 0) *D.step = j + 1;
}

// the coefficients of steps j0 .. j0+nn-1 of every problem of a batch into one buffer (one copy to the
// host per chunk): per problem nn alpha, nn h_{j+1,j}, nn h_{j,j+1} (z64), then nn flags
__global__ void __launch_bounds__(64) qb_gather_coef(const LzScalars *S, int j0, int nn, char *out)
{
    const LzScalars &L = S[blockIdx.x];
    if (!L.alpha) return;  // a problem with y = 0 has no scalar table
    const size_t per = 3 * sizeof(z64) * (size_t)nn + sizeof(int) * (size_t)nn;
    z64 *o = reinterpret_cast<z64 *>(out + per * blockIdx.x);
    int *f = reinterpret_cast<int *>(o + 3 * nn);
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
        o[i] = L.alpha[j0 + i];
        o[nn + i] = L.hsub[j0 + i];
        o[2 * nn + i] = L.hsup[j0 + i];
        f[i] = L.flag[j0 + i];
    }
}

class QmrBatch {
  public:
    QmrBatch(const sgn_problem *pb, int np, const sgn_rational &rf, const sgn_ms_opts &o, hipStream_t s)
        : o_(o), s_(s)
    {
        for (int k = 0; k < np; ++k) pr_.push_back(std::make_unique<QmrSolve>(pb[k], rf, o, s, &next_));
        ctx_ = pr_.empty() ? nullptr : &pr_[0]->ctx_;
        for (auto &p : pr_) SGN_REQUIRE(&p->ctx_ == ctx_, "multishift_qmr: problems of one call need one context");
    }
    ~QmrBatch()
    {
        drop_graph();
        for (QbDesc *d : ddesc_)
            if (d) (void)hipFree(d);
        if (dcoef_) (void)hipFree(dcoef_);
        if (hcoef_) (void)hipHostFree(hcoef_);
    }
    sgn_status run(sgn_stats *st);

  private:
    std::vector<std::unique_ptr<QmrSolve>> pr_;
    std::map<size_t, size_t> next_;  // basis slots handed out from the context's pools, per vector size
    const sgn_ms_opts &o_;
    hipStream_t s_;
    Context *ctx_ = nullptr;
    std::vector<int> group_[3];  // problems of each stencil precision still stepping
    std::vector<bool> active_;
    QbDesc *ddesc_[3] = {nullptr, nullptr, nullptr};
    size_t dcap_[3] = {0, 0, 0};
    StencilBatch stb_[3][4];
    int nvb_max_[3] = {0, 0, 0};
    hipGraphExec_t gexec_ = nullptr;
    // the chunk's coefficients of every problem: scalar tables and a gather buffer (device), and
    // the pinned host mirror
    char *dcoef_ = nullptr, *hcoef_ = nullptr;

    static int phase_of(const QmrSolve &q) { return !q.f32_ ? 0 : (q.sp_ == SGN_PREC_F32 ? 1 : 2); }
    void drop_graph()
    {
        if (gexec_) (void)hipGraphExecDestroy(gexec_);
        gexec_ = nullptr;
    }
    void rebuild();
    void launch_step(hipStream_t strm);
    void iterate(int count);
};

void QmrBatch::rebuild()
{
    drop_graph();
    for (auto &g : group_) g.clear();
    for (int k = 0; k < (int)pr_.size(); ++k)
        if (active_[k]) group_[phase_of(*pr_[k])].push_back(k);
    for (int ph = 0; ph < 3; ++ph) {
        const std::vector<int> &g = group_[ph];
        std::vector<StencilJob> jobs[4];
        std::vector<QbDesc> desc(g.size());
        nvb_max_[ph] = 0;
        for (size_t j = 0; j < g.size(); ++j) {
            QmrSolve &q = *pr_[g[j]];
            const bool f = ph >= 1;
            void *vin = f ? q.v32_->p : q.vcur_->p, *win = f ? q.w32_->p : q.wcur_->p;
            void *t = f ? q.t32_->p : q.tmp_->p, *u = f ? q.u32_->p : q.u_->p, *z = f ? q.z32_->p : q.z_->p;
            jobs[0].push_back(StencilJob{&q.lat_, q.opA_, vin, t, Epilogue{}});
            StencilJob j2{&q.lat_, q.opA_, t, u, Epilogue{}};  // u = c^2 H (H vh_j), partials of wh_j^H u
            j2.ep.a = q.c2_;
            j2.ep.w = win;
            j2.ep.partials = q.part1_;
            jobs[1].push_back(j2);
            jobs[2].push_back(StencilJob{&q.lat_, q.opAh_, win, t, Epilogue{}});
            StencilJob j4{&q.lat_, q.opAh_, t, z, Epilogue{}};  // z = c^2 H^H (H^H wh_j)
            j4.ep.a = q.c2_;
            jobs[3].push_back(j4);
            char *wb = static_cast<char *>(q.Wb_->p);
            desc[j] = QbDesc{q.S_, q.dstep_, q.ddone_, nullptr,
                             {(double2 *)wb, (double2 *)(wb + q.i64_), (double2 *)(wb + 2 * q.i64_)},
                             (double2 *)q.vcur_->p, (double2 *)q.wcur_->p, (float4 *)(f ? q.v32_->p : nullptr),
                             (float4 *)(f ? q.w32_->p : nullptr), u, z, q.part1_, q.part2_, 0, (int)q.Sst_};
            nvb_max_[ph] = std::max(nvb_max_[ph], q.nvb_);
        }
        const sgn_prec sp = ph == 0 ? SGN_PREC_F64 : (ph == 1 ? SGN_PREC_F32 : SGN_PREC_F32_H16);
        for (int k = 0; k < 4; ++k) stb_[ph][k].prepare(jobs[k], sp);
        if (g.empty()) continue;
        for (size_t j = 0; j < g.size(); ++j) {
            QmrSolve &q = *pr_[g[j]];
            desc[j].nb1 = stb_[ph][1].blocks(j);
            desc[j].slots = q.dslots_;
        }
        const size_t need = sizeof(QbDesc) * g.size();
        if (need > dcap_[ph]) {
            if (ddesc_[ph]) SGN_HIP(hipFree(ddesc_[ph]));
            ddesc_[ph] = nullptr;
            dcap_[ph] = 0;
            if (hipMalloc(&ddesc_[ph], need) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "multishift_qmr: batch"};
            dcap_[ph] = need;
        }
        SGN_HIP(hipMemcpy(ddesc_[ph], desc.data(), need, hipMemcpyHostToDevice));
    }
}

void QmrBatch::launch_step(hipStream_t strm)
{
    for (int ph = 0; ph < 3; ++ph) {
        const int np = (int)group_[ph].size();
        if (!np) continue;
        const QbDesc *d = ddesc_[ph];
        stb_[ph][0].launch(strm);
        stb_[ph][1].launch(strm);
        hipLaunchKernelGGL(qb_alpha_batch, dim3(np), dim3(256), 0, strm, d);
        stb_[ph][2].launch(strm);
        stb_[ph][3].launch(strm);
        if (ph >= 1)
            hipLaunchKernelGGL(qb_update_batch<true>, dim3(nvb_max_[ph], np), dim3(256), 0, strm, d);
        else
            hipLaunchKernelGGL(qb_update_batch<false>, dim3(nvb_max_[ph], np), dim3(256), 0, strm, d);
        hipLaunchKernelGGL(qb_step_batch, dim3(np), dim3(256), 0, strm, d, nvb_max_[ph]);
    }
    SGN_HIP(hipGetLastError());
}

void QmrBatch::iterate(int count)
{
    replay_or_capture(*ctx_, gexec_, true, s_, [&](hipStream_t strm) {
        for (int it = 0; it < count; ++it) launch_step(strm);
    });
}

sgn_status QmrBatch::run(sgn_stats *st)
{
    if (pr_.empty()) return SGN_OK;
    SGN_HIP(hipSetDevice(ctx_->device));
    active_.assign(pr_.size(), false);
    int nactive = 0;
    for (size_t k = 0; k < pr_.size(); ++k) {
        active_[k] = pr_[k]->setup(st ? st + k : nullptr, true);
        nactive += active_[k] ? 1 : 0;
    }
    const int poll = pr_[0]->poll_;
    const int np = (int)pr_.size();
    const size_t per = 3 * sizeof(z64) * (size_t)poll + sizeof(int) * (size_t)poll;
    {
        std::vector<LzScalars> tab(np);
        for (int k = 0; k < np; ++k) tab[k] = pr_[k]->S_;
        if (hipMalloc(&dcoef_, sizeof(LzScalars) * np + per * np) != hipSuccess) {
            dcoef_ = nullptr;
            throw Failure{SGN_ERR_NOMEM, "multishift_qmr: batch"};
        }
        SGN_HIP(hipMemcpy(dcoef_, tab.data(), sizeof(LzScalars) * np, hipMemcpyHostToDevice));
        SGN_HIP(hipHostMalloc(reinterpret_cast<void **>(&hcoef_), per * np));
    }
    const LzScalars *dtab = reinterpret_cast<const LzScalars *>(dcoef_);
    char *dbuf = dcoef_ + sizeof(LzScalars) * np;
    int launched = 0, finished_since = 0, in_launch = 0;
    bool dirty = true;
    const int one = 1;
    while (nactive > 0) {
        // every problem in the launch takes `poll` more steps (a finished one only idles: its
        // kernels see its done flag)
        int maxit = 0;
        for (size_t k = 0; k < pr_.size(); ++k)
            if (active_[k]) maxit = std::max(maxit, pr_[k]->maxiter_);
        const int chunk = std::min(poll, maxit - launched);
        for (size_t k = 0; k < pr_.size(); ++k)
            if (active_[k]) pr_[k]->ensure_slots(launched + chunk);
        if (dirty || chunk != poll) {
            rebuild();
            dirty = false;
            finished_since = 0;
            in_launch = nactive;
        }
        iterate(chunk);
        const int j0 = launched;
        launched += chunk;
        // every problem's coefficients of the chunk in one copy (problems with y = 0 have no scalar
        // table and are skipped by the kernel; only active problems' entries are read)
        const size_t pc = 3 * sizeof(z64) * (size_t)chunk + sizeof(int) * (size_t)chunk;
        hipLaunchKernelGGL(qb_gather_coef, dim3(np), dim3(64), 0, s_, dtab, j0, chunk, dbuf);
        SGN_HIP(hipGetLastError());
        SGN_HIP(hipMemcpyAsync(hcoef_, dbuf, pc * np, hipMemcpyDeviceToHost, s_));
        SGN_HIP(hipStreamSynchronize(s_));
        for (size_t k = 0; k < pr_.size(); ++k) {
            if (!active_[k]) continue;
            QmrSolve &q = *pr_[k];
            const z64 *o = reinterpret_cast<const z64 *>(hcoef_ + pc * k);
            const int *f = reinterpret_cast<const int *>(o + 3 * chunk);
            for (int i = 0; i < chunk; ++i) {
                q.halpha_[j0 + i] = o[i];
                q.hsub_[j0 + i] = o[chunk + i];
                q.hsup_[j0 + i] = o[2 * chunk + i];
                q.hflag_[j0 + i] = f[i];
            }
            if (q.absorb_host(j0, std::min(launched, q.maxiter_))) {
                active_[k] = false;
                --nactive;
                ++finished_since;
                SGN_HIP(hipMemcpyAsync(q.ddone_, &one, sizeof(int), hipMemcpyHostToDevice, s_));
            } else if (q.switch_precision()) {
                dirty = true;
            }
        }
        SGN_HIP(hipStreamSynchronize(s_));  // the done flags are written before the next replay
        if (nactive > 0 && 4 * finished_since >= in_launch) dirty = true;
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

extern "C" sgn_status multishift_qmr(const sgn_problem *pb, int nprob, const sgn_rational *rf, const sgn_ms_opts *o,
                                     sgn_stats *stats, void *stream)
{
    sgn_status worst = SGN_OK;
    const sgn_status st = guard([&] {
        SGN_REQUIRE(pb && rf && o && nprob >= 0, "multishift_qmr: null argument");
        SGN_REQUIRE(rf->s >= 1 && rf->s <= SGN_MAX_POLES, "multishift_qmr: bad number of poles");
        SGN_REQUIRE(rf->c > 0 && std::isfinite(rf->c), "multishift_qmr: bad scale c");
        for (int i = 0; i < rf->s; ++i)
            SGN_REQUIRE(rf->sigma[i] < 0 && std::isfinite(rf->omega[i]), "multishift_qmr: shifts must be negative");
        SGN_REQUIRE(o->tol > 0 && o->tol < 1, "multishift_qmr: tol must be in (0, 1)");
        SGN_REQUIRE(o->basis_slots >= 0, "multishift_qmr: the basis is always stored (basis_slots >= 0)");
        SGN_REQUIRE(o->prec == SGN_PREC_F64 || o->prec == SGN_PREC_F32 || o->prec == SGN_PREC_F32_H16,
                    "multishift_qmr: bad precision");
        for (int p = 0; p < nprob; ++p) {
            SGN_REQUIRE(pb[p].lat && pb[p].b && pb[p].x, "multishift_qmr: null problem field");
            SGN_REQUIRE(std::isfinite(pb[p].mu), "multishift_qmr: mu not finite");
        }
        if (nprob > 1) {  // the problems in lockstep
            QmrBatch batch(pb, nprob, *rf, *o, static_cast<hipStream_t>(stream));
            worst = batch.run(stats);
            return;
        }
        for (int p = 0; p < nprob; ++p) {
            QmrSolve solver(pb[p], *rf, *o, static_cast<hipStream_t>(stream));
            const sgn_status r = solver.run(stats ? stats + p : nullptr);
            if (r != SGN_OK && worst == SGN_OK) worst = r;
        }
    });
    return st != SGN_OK ? st : worst;
}
