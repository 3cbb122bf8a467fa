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
#include <chrono>
#include <complex>
#include <vector>

#include "field_io.h"
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

__global__ void lz_alpha_kernel(const z64 *partials, int nblk, LzScalars S, int j)
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

__global__ void lz_step_kernel(const z64 *partials, int nblk, LzScalars S, int j, double tol)
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

__device__ __forceinline__ z64 ld2(const double2 *p, int64_t i)
{
    double2 t = p[i];
    return {t.x, t.y};
}

// One thread per pair of complex entries (e0 = 2*c2*V + s, e1 = e0 + V) so that
// the FP32 stencil outputs ([6][V] float4) and FP64 vectors line up.
template <bool F32>
__global__ void __launch_bounds__(256) lz_update_kernel(const void *u_, const void *z_, const double2 *vj,
                                                        const double2 *vjm, const double2 *wj, const double2 *wjm,
                                                        double2 *vn, double2 *wn, float4 *vn32, float4 *wn32,
                                                        LzScalars S, int j, int V /* component stride */,
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
    PooledBasis(Context &c, size_t b, size_t cap_, const char *w) : ctx(c), bytes(b), cap(cap_), who(w) {}
    void *operator[](int j) const { return slots[j]; }
    void ensure(int upto)  // slots 0 .. upto exist
    {
        auto &pool = ctx.basis_pools[bytes];
        while ((int)slots.size() <= upto) {
            const size_t idx = slots.size();
            if (idx >= cap) throw Failure{SGN_ERR_NOMEM, std::string(who) + ": Krylov basis exceeds its slot budget"};
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
                                   (double2 *)Wj(j + 1), (float4 *)v32.p, (float4 *)w32.p, S, j, (int)Sst, part);
            else
                hipLaunchKernelGGL(lz_update_kernel<false>, dim3(nvb), dim3(256), 0, s, u.p, z.p,
                                   (const double2 *)Vj(j), vjm, (const double2 *)Wj(j), wjm, (double2 *)vn,
                                   (double2 *)Wj(j + 1), (float4 *)nullptr, (float4 *)nullptr, S, j, (int)Sst, part);
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

sgn_status qmr_one(const sgn_problem &pb, const sgn_rational &rf, const sgn_ms_opts &o, sgn_stats *st, hipStream_t s)
{
    const auto t_start = std::chrono::steady_clock::now();
    Lattice &lat = *as_lattice(pb.lat);
    Context &ctx = *lat.ctx;
    SGN_HIP(hipSetDevice(ctx.device));
    const int64_t V = lat.V, Sst = lat.S, nc = 12 * V, ni = 12 * Sst;
    const size_t b64 = (size_t)nc * 16, i64 = (size_t)ni * 16, b32 = (size_t)ni * 8;
    // precision schedule: FP64 steps while the largest quasi-residual is above theta32 ||y||,
    // then the stencil in FP32 (and with FP16 links below theta16 ||y|| for SGN_PREC_F32_H16);
    // the recurrences and the basis stay FP64
    const bool mixed = o.prec != SGN_PREC_F64;
    const double theta32 = mixed ? (o.theta32 > 0 ? o.theta32 : 1e-3) : 0.0;
    const double theta16 = o.prec == SGN_PREC_F32_H16 ? (o.theta16 > 0 ? o.theta16 : 1e-6) : 0.0;
    sgn_prec sp = SGN_PREC_F64;
    bool f32 = false;
    const int ns = rf.s;
    const double c2 = rf.c * rf.c;
    const int maxiter = o.maxiter > 0 ? o.maxiter : 10000;
    const int poll = o.poll > 0 ? o.poll : 4;
    if (st) {
        *st = sgn_stats{};
        st->nshift = ns;
    }
    OpSpec opA, opAh;
    opA.mu = pb.mu;
    opAh.mu = -pb.mu;

    // x <- x_P, y = c H (I - P) b
    DevBuf rcan(b64), y(i64), tmp(i64);
    deflation_prologue(ctx, pb.defl, nc, pb.b, pb.x, rcan.p, nullptr, s);
    pack_spinor(lat, rcan.p, tmp.p, SGN_PREC_F64, s);
    {
        Epilogue ep;
        ep.a = rf.c;
        dslash_launch(lat, SGN_PREC_F64, opA, tmp.p, y.p, ep, s);
    }
    const double ynorm = norm_sync(ctx, y.p, ni, false, s);
    SGN_REQUIRE(std::isfinite(ynorm), "multishift_qmr: b contains NaN or Inf");
    if (ynorm == 0.0) {  // x = x_P
        if (pb.x_shift)
            for (int i = 0; i < ns; ++i)
                if (pb.x_shift[i]) SGN_HIP(hipMemsetAsync(pb.x_shift[i], 0, b64, s));
        SGN_HIP(hipStreamSynchronize(s));
        return SGN_OK;
    }

    // stored basis: slot j holds vh_j (FP64, internal layout), from the context's pool
    size_t cap;
    if (o.basis_slots > 0) {
        cap = (size_t)o.basis_slots;
    } else {
        size_t fr = 0, tot = 0;
        SGN_HIP(hipMemGetInfo(&fr, &tot));
        cap = ctx.basis_pools[i64].size() + fr / 2 / i64;
    }
    PooledBasis basis(ctx, i64, cap, "multishift_qmr");
    basis.ensure(0);
    DevBuf Wb(3 * i64), u(i64), z(i64);
    DevBuf v32(mixed ? b32 : 0), w32(mixed ? b32 : 0), t32(mixed ? b32 : 0), u32(mixed ? b32 : 0),
        z32(mixed ? b32 : 0);
    const size_t nscal = sizeof(z64) * (5 * (size_t)maxiter + 2) + sizeof(int) * maxiter;
    DevBuf scal(nscal);
    LzScalars S;
    S.alpha = scal.as<z64>();
    S.hsub = S.alpha + maxiter;
    S.hsup = S.hsub + maxiter;
    S.sv = S.hsup + maxiter;
    S.tw = S.sv + (maxiter + 1);
    S.flag = reinterpret_cast<int *>(S.tw + (maxiter + 1));
    auto Wj = [&](int j) { return static_cast<char *>(Wb.p) + (size_t)(j % 3) * i64; };
    const z64 s0 = {1.0 / ynorm, 0.0};  // v_1 = s_0 y,  w_1 = t_0 y = v_1
    SGN_HIP(hipMemsetAsync(scal.p, 0, nscal, s));
    SGN_HIP(hipMemcpyAsync(S.sv, &s0, sizeof(z64), hipMemcpyHostToDevice, s));
    SGN_HIP(hipMemcpyAsync(S.tw, &s0, sizeof(z64), hipMemcpyHostToDevice, s));
    SGN_HIP(hipMemcpyAsync(basis[0], y.p, i64, hipMemcpyDeviceToDevice, s));
    SGN_HIP(hipMemcpyAsync(Wj(0), y.p, i64, hipMemcpyDeviceToDevice, s));
    const int nst = dslash_blocks(lat);
    const int nvb = vec_blocks(6 * Sst);
    z64 *part = static_cast<z64 *>(ctx.ensure_partials(sizeof(z64) * std::max(nst, 2 * nvb)));

    // one Lanczos step on A': alpha_j, vh_{j+1}, wh_{j+1}, h_{j+1,j}, h_{j,j+1}
    auto step = [&](int j) {
        dslash_launch(lat, sp, opA, f32 ? v32.p : basis[j], f32 ? t32.p : tmp.p, Epilogue{}, s);
        Epilogue ep;  // u = c^2 H (H vh_j), partials of wh_j^H u
        ep.a = c2;
        ep.w = f32 ? w32.p : Wj(j);
        ep.partials = part;
        const int nb1 = dslash_launch(lat, sp, opA, f32 ? t32.p : tmp.p, f32 ? u32.p : u.p, ep, s);
        hipLaunchKernelGGL(lz_alpha_kernel, dim3(1), dim3(256), 0, s, part, nb1, S, j);
        dslash_launch(lat, sp, opAh, f32 ? w32.p : Wj(j), f32 ? t32.p : tmp.p, Epilogue{}, s);
        Epilogue ez;  // z = c^2 H^H (H^H wh_j)
        ez.a = c2;
        dslash_launch(lat, sp, opAh, f32 ? t32.p : tmp.p, f32 ? z32.p : z.p, ez, s);
        const double2 *vjm = j > 0 ? static_cast<const double2 *>(basis[j - 1]) : nullptr;
        const double2 *wjm = j > 0 ? reinterpret_cast<const double2 *>(Wj(j - 1)) : nullptr;
        const int pr = ctx.prof_start(s, SGN_K_SEED_UPDATE);
        if (f32)
            hipLaunchKernelGGL(lz_update_kernel<true>, dim3(nvb), dim3(256), 0, s, u32.p, z32.p,
                               (const double2 *)basis[j], vjm, (const double2 *)Wj(j), wjm, (double2 *)basis[j + 1],
                               (double2 *)Wj(j + 1), (float4 *)v32.p, (float4 *)w32.p, S, j, (int)Sst, part);
        else
            hipLaunchKernelGGL(lz_update_kernel<false>, dim3(nvb), dim3(256), 0, s, u.p, z.p,
                               (const double2 *)basis[j], vjm, (const double2 *)Wj(j), wjm, (double2 *)basis[j + 1],
                               (double2 *)Wj(j + 1), (float4 *)nullptr, (float4 *)nullptr, S, j, (int)Sst, part);
        const double io = (f32 ? 2.0 * b32 : 2.0 * i64) + (j > 0 ? 4.0 : 2.0) * i64 + 2.0 * i64 + (f32 ? 2.0 * b32 : 0.0);
        ctx.prof_stop(pr, s, SGN_K_SEED_UPDATE, io, 40.0 * ni);
        hipLaunchKernelGGL(lz_step_kernel, dim3(1), dim3(256), 0, s, part, nvb, S, j, 1e-14);
        SGN_HIP(hipGetLastError());
    };

    std::vector<QmrShift> G(ns);
    for (int i = 0; i < ns; ++i) {
        G[i].sigma = rf.sigma[i];
        G[i].g.assign(1, cplx(ynorm, 0.0));
    }
    std::vector<z64> halpha(maxiter), hsub(maxiter), hsup(maxiter);
    std::vector<int> hflag(maxiter);
    sgn_status result = SGN_OK;
    double small_ms = 0.0;
    int launched = 0, kused = -1;
    const auto t_kry = std::chrono::steady_clock::now();
    while (kused < 0) {
        const int chunk = std::min(poll, maxiter - launched);
        basis.ensure(launched + chunk);
        for (int q = 0; q < chunk; ++q) step(launched + q);
        const int j0 = launched;
        launched += chunk;
        const int nn = launched - j0;
        SGN_HIP(hipMemcpyAsync(halpha.data() + j0, S.alpha + j0, sizeof(z64) * nn, hipMemcpyDeviceToHost, s));
        SGN_HIP(hipMemcpyAsync(hsub.data() + j0, S.hsub + j0, sizeof(z64) * nn, hipMemcpyDeviceToHost, s));
        SGN_HIP(hipMemcpyAsync(hsup.data() + j0, S.hsup + j0, sizeof(z64) * nn, hipMemcpyDeviceToHost, s));
        SGN_HIP(hipMemcpyAsync(hflag.data() + j0, S.flag + j0, sizeof(int) * nn, hipMemcpyDeviceToHost, s));
        SGN_HIP(hipStreamSynchronize(s));
        const auto t0 = std::chrono::steady_clock::now();
        for (int j = j0; j < launched; ++j) {
            const cplx al(halpha[j].r, halpha[j].i), hp = j > 0 ? cplx(hsup[j - 1].r, hsup[j - 1].i) : cplx(0.0);
            double tmax = 0.0;
            for (auto &g : G) {
                if (!g.add_column(j, hp, al, hsub[j].r))
                    throw Failure{SGN_ERR_BREAKDOWN, "multishift_qmr: singular shifted tridiagonal"};
                tmax = std::max(tmax, g.tau());
            }
            if (!std::isfinite(tmax))
                throw Failure{SGN_ERR_BREAKDOWN, "multishift_qmr: non-finite Lanczos coefficients"};
            if (tmax <= o.tol * ynorm || hsub[j].r == 0.0) {  // converged, or invariant subspace (exact)
                kused = j + 1;
                break;
            }
            if (hflag[j])
                throw Failure{SGN_ERR_BREAKDOWN, "two-sided Lanczos breakdown at step " + std::to_string(j + 1)};
        }
        small_ms += ms_since(t0);
        if (kused < 0 && launched >= maxiter) {
            kused = launched;
            result = SGN_ERR_NOT_CONVERGED;
        }
        if (kused < 0 && mixed) {
            double tmax = 0.0;
            for (const auto &g : G) tmax = std::max(tmax, g.tau());
            if (!f32 && tmax < theta32 * ynorm) {  // FP32 copies of the current vh_j, wh_j
                convert_64_to_32(basis[launched], v32.p, Sst, s);
                convert_64_to_32(Wj(launched), w32.p, Sst, s);
                f32 = true;
                sp = SGN_PREC_F32;
            }
            if (f32 && sp == SGN_PREC_F32 && tmax < theta16 * ynorm) sp = SGN_PREC_F32_H16;
        }
    }
    const double kry_ms = ms_since(t_kry);

    // coefficients of the stored vectors: x_i = sum_j z_ij s_j vh_j
    std::vector<z64> hsv(kused);
    SGN_HIP(hipMemcpy(hsv.data(), S.sv, sizeof(z64) * kused, hipMemcpyDeviceToHost));
    std::vector<std::vector<cplx>> Z(ns);
    for (int i = 0; i < ns; ++i) Z[i] = G[i].solve(kused);
    // coefficient sets: 0 = sum_i omega_i x_i, then one per shift whose x_i is requested or
    // verified; all are uploaded before the first lift is queued (no buffer is reused)
    std::vector<int> sel;
    for (int i = 0; i < ns; ++i)
        if ((pb.x_shift && pb.x_shift[i]) || o.verify) sel.push_back(i);
    const size_t nset = 1 + sel.size();
    std::vector<z64> hcoef(nset * kused);
    for (int j = 0; j < kused; ++j) {
        cplx d = 0.0;
        for (int i = 0; i < ns; ++i) d += rf.omega[i] * Z[i][j];
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
        basis.lift(dcoef.as<z64>() + set * kused, static_cast<const void *const *>(dtab.p), kused, ni, out, s);
        ctx.prof_stop(pr, s, SGN_K_LIFT, (double)i64 * (kused + 1), 8.0 * ni * kused);
    };
    // canonical v <- (I - P) v (rounding components along the deflated eigenvectors)
    const bool deflated = pb.defl && pb.defl->m > 0;
    DevBuf dfc(deflated ? sizeof(z64) * pb.defl->m : 0);
    auto project_out = [&](void *v) {
        if (!deflated) return;
        deflate_dots(pb.defl->L, pb.defl->m, v, nc, dfc.as<z64>(), ctx, s);
        deflate_combine(v, {1.0, 0.0}, {-1.0, 0.0}, pb.defl->R, pb.defl->m, dfc.as<z64>(), nullptr, nc, s);
    };
    lift(0, tmp.p);
    unpack_spinor(lat, tmp.p, rcan.p, SGN_PREC_F64, s);
    project_out(rcan.p);
    axpby64({1.0, 0.0}, rcan.p, {1.0, 0.0}, pb.x, nc, s);

    // per-shift solutions: requested ones, and all of them for the FP64 residual check
    std::vector<double> res(ns);
    for (int i = 0; i < ns; ++i) res[i] = G[i].tau() / ynorm;
    int extra_mv = 0;
    DevBuf h(o.verify ? i64 : 0), q(o.verify ? i64 : 0);
    for (size_t k = 0; k < sel.size(); ++k) {
        const int i = sel[k];
        lift(k + 1, tmp.p);
        if (o.verify) {  // r_i = y - (c^2 H^2 - sigma_i) x_i in FP64
            dslash_launch(lat, SGN_PREC_F64, opA, tmp.p, h.p, Epilogue{}, s);
            Epilogue ep;
            ep.a = -c2;
            ep.z = tmp.p;
            ep.b = {rf.sigma[i], 0.0};
            dslash_launch(lat, SGN_PREC_F64, opA, h.p, q.p, ep, s);
            axpby64({1.0, 0.0}, y.p, {1.0, 0.0}, q.p, ni, s);
            res[i] = norm_sync(ctx, q.p, ni, false, s) / ynorm;
            extra_mv += 2;
        }
        if (pb.x_shift && pb.x_shift[i]) {
            unpack_spinor(lat, tmp.p, pb.x_shift[i], SGN_PREC_F64, s);
            project_out(pb.x_shift[i]);
        }
    }
    SGN_HIP(hipStreamSynchronize(s));
    if (st) {
        st->iterations = kused;
        st->matvecs = 4 * launched + 1 + extra_mv;
        double mx = 0.0;
        for (int i = 0; i < ns; ++i) {
            st->shift_residual[i] = res[i];
            mx = std::max(mx, res[i]);
        }
        st->residual = mx;
        st->krylov_ms = kry_ms;
        st->small_ms = small_ms;
        st->total_ms = ms_since(t_start);
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
        for (int p = 0; p < nprob; ++p) {
            const sgn_status r = qmr_one(pb[p], *rf, *o, stats ? stats + p : nullptr, static_cast<hipStream_t>(stream));
            if (r != SGN_OK && worst == SGN_OK) worst = r;
        }
    });
    return st != SGN_OK ? st : worst;
}
