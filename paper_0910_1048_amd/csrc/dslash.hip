// Wilson-Dirac stencil H_W(mu) = gamma5 D_W(mu) on gfx950.
//
// One thread per lattice site, 256 threads (4 wavefronts) per block, blocks
// ordered per XCD (xcd_block).  Each of the 8 hops projects the neighbour
// spinor to a half spinor with (1 -+ gamma_nu) (DeGrand-Rossi basis), applies
// U or U^H to the two colour vectors, scales by -kappa * weight * boundary
// factor, and adds the reconstructed 4-spinor.  The chemical potential enters
// only as the weights e^{-mu} (forward time hop) and e^{+mu} (backward time
// hop); the adjoint H_W(mu)^H = H_W(-mu) is the same kernel with mu -> -mu.
// Single-RHS stencil: HBM-bound, 1368 flop per site.
#include "field_io.h"

#ifndef SGN_STENCIL_WAVES
#define SGN_STENCIL_WAVES 1
#endif

namespace sgn {

namespace {

struct StencilParams {
    const void *in;
    void *out;
    const void *links;
    int V;
    int L[4];
    int stride[4];
    float bcf[4];       // boundary factor per direction (hops that wrap)
    double kappa;
    double wf_t, wb_t;  // time-hop weights e^{-mu}, e^{+mu}
    float s5_in;        // -1: apply gamma5 to the input first
    float s5_out;       // -1: apply gamma5 to the result
    // epilogue
    double a;
    z64 b;
    const z64 *b_dev;
    const void *z;
    const void *w;
    z64 *partials;
    const z64 *in_scale;
};

// Half-spinor projection (1 - gamma_nu) for FWD, (1 + gamma_nu) otherwise:
// h[0..2] = colour vector of the upper-spin-0 row, h[3..5] = spin-1 row.
template <int NU, bool FWD, typename R>
__device__ __forceinline__ void project(const cpx<R> p[12], cpx<R> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if constexpr (NU == 0) {
            h[c] = FWD ? p0 + times_mi(p3) : p0 + times_i(p3);
            h[3 + c] = FWD ? p1 + times_mi(p2) : p1 + times_i(p2);
        } else if constexpr (NU == 1) {
            h[c] = FWD ? p0 + p3 : p0 - p3;
            h[3 + c] = FWD ? p1 - p2 : p1 + p2;
        } else if constexpr (NU == 2) {
            h[c] = FWD ? p0 + times_mi(p2) : p0 + times_i(p2);
            h[3 + c] = FWD ? p1 + times_i(p3) : p1 + times_mi(p3);
        } else {
            h[c] = FWD ? p0 - p2 : p0 + p2;
            h[3 + c] = FWD ? p1 - p3 : p1 + p3;
        }
    }
}

// acc += coef * reconstruct(chi): upper spins are chi0, chi1; lower spins follow
// from the rank-2 structure of (1 -+ gamma_nu).
template <int NU, bool FWD, typename R>
__device__ __forceinline__ void accumulate(cpx<R> acc[12], const cpx<R> chi[6], R coef)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<R> h0 = coef * chi[c], h1 = coef * chi[3 + c];
        acc[c] = acc[c] + h0;
        acc[3 + c] = acc[3 + c] + h1;
        cpx<R> r2, r3;
        if constexpr (NU == 0) {
            r2 = FWD ? times_i(h1) : times_mi(h1);
            r3 = FWD ? times_i(h0) : times_mi(h0);
        } else if constexpr (NU == 1) {
            r2 = FWD ? -h1 : h1;
            r3 = FWD ? h0 : -h0;
        } else if constexpr (NU == 2) {
            r2 = FWD ? times_i(h0) : times_mi(h0);
            r3 = FWD ? times_mi(h1) : times_i(h1);
        } else {
            r2 = FWD ? -h0 : h0;
            r3 = FWD ? -h1 : h1;
        }
        acc[6 + c] = acc[6 + c] + r2;
        acc[9 + c] = acc[9 + c] + r3;
    }
}

// chi = U h (forward) or U^H h (backward), on both colour vectors
template <bool ADJ, typename R>
__device__ __forceinline__ void link_mul(const cpx<R> u[9], const cpx<R> h[6], cpx<R> chi[6])
{
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<R> s = {0, 0};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if constexpr (ADJ)
                    s = s + cmulc(u[b * 3 + a], h[3 * v + b]);
                else
                    s = s + u[a * 3 + b] * h[3 * v + b];
            }
            chi[3 * v + a] = s;
        }
}

template <typename R>
using SpT = typename SpinorStore<R>::type;

// Ordering fence between hops: the accumulator must be complete here and no
// later load may move above it.  Without it the compiler issues all 8
// neighbour gathers up front and the kernel needs >300 VGPRs (spills, one
// wave per SIMD).
template <typename R>
__device__ __forceinline__ void pin(cpx<R> acc[12])
{
#pragma unroll
    for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(acc[k].r), "+v"(acc[k].i)::"memory");
}

template <int NU, typename R, typename LT>
__device__ __forceinline__ void hop_pair(cpx<R> acc[12], const StencilParams &P, int s, int coord, R s5)
{
    const SpT<R> *in = static_cast<const SpT<R> *>(P.in);
    const LT *U = static_cast<const LT *>(P.links);
    const int L = P.L[NU], st = P.stride[NU];
    const R kap = static_cast<R>(P.kappa);
    R wf = 1, wb = 1;
    if constexpr (NU == 3) {
        wf = static_cast<R>(P.wf_t);
        wb = static_cast<R>(P.wb_t);
    }
    cpx<R> p[12], h[6], chi[6], u[9];
    // forward hop: (1 - gamma) U_nu(x) psi(x + nu)
    {
        const bool wrap = coord == L - 1;
        const int n = wrap ? s - (L - 1) * st : s + st;
        load_spinor(in, P.V, n, p);
#pragma unroll
        for (int k = 6; k < 12; ++k) p[k] = s5 * p[k];
        project<NU, true>(p, h);
        load_link<R>(U, P.V, NU, s, u);
        link_mul<false>(u, h, chi);
        const R coef = -kap * wf * (wrap ? static_cast<R>(P.bcf[NU]) : R(1));
        accumulate<NU, true>(acc, chi, coef);
    }
    pin(acc);
    // backward hop: (1 + gamma) U_nu(x - nu)^H psi(x - nu)
    {
        const bool wrap = coord == 0;
        const int n = wrap ? s + (L - 1) * st : s - st;
        load_spinor(in, P.V, n, p);
#pragma unroll
        for (int k = 6; k < 12; ++k) p[k] = s5 * p[k];
        project<NU, false>(p, h);
        load_link<R>(U, P.V, NU, n, u);
        link_mul<true>(u, h, chi);
        const R coef = -kap * wb * (wrap ? static_cast<R>(P.bcf[NU]) : R(1));
        accumulate<NU, false>(acc, chi, coef);
    }
    pin(acc);
}

template <typename R, typename LT, bool kEpi, bool kDot>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SGN_STENCIL_WAVES))) stencil_kernel(StencilParams P)
{
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = blk * 256 + threadIdx.x;
    const bool valid = s < P.V;
    double dr = 0.0, di = 0.0;
    if (valid) {
        int c0 = s % P.L[0];
        int q = s / P.L[0];
        int c1 = q % P.L[1];
        q /= P.L[1];
        int c2 = q % P.L[2];
        int c3 = q / P.L[2];
        const R s5 = static_cast<R>(P.s5_in);
        cpx<R> acc[12];
        load_spinor(static_cast<const SpT<R> *>(P.in), P.V, s, acc);
#pragma unroll
        for (int k = 6; k < 12; ++k) acc[k] = s5 * acc[k];
        hop_pair<0, R, LT>(acc, P, s, c0, s5);
        hop_pair<1, R, LT>(acc, P, s, c1, s5);
        hop_pair<2, R, LT>(acc, P, s, c2, s5);
        hop_pair<3, R, LT>(acc, P, s, c3, s5);
        const R s5o = static_cast<R>(P.s5_out);
#pragma unroll
        for (int k = 6; k < 12; ++k) acc[k] = s5o * acc[k];
        if constexpr (kEpi) {
            cpx<R> sc = {static_cast<R>(P.a), R(0)};
            if (P.in_scale) {
                z64 t = *P.in_scale;
                sc = {static_cast<R>(P.a * t.r), static_cast<R>(P.a * t.i)};
            }
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = sc * acc[k];
            if (P.z) {
                z64 bb = P.b;
                if (P.b_dev) {
                    z64 t = *P.b_dev;
                    bb = {bb.r * t.r - bb.i * t.i, bb.r * t.i + bb.i * t.r};
                }
                cpx<R> b = {static_cast<R>(bb.r), static_cast<R>(bb.i)};
                cpx<R> zz[12];
                load_spinor(static_cast<const SpT<R> *>(P.z), P.V, s, zz);
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = acc[k] + b * zz[k];
            }
        }
        store_spinor(static_cast<SpT<R> *>(P.out), P.V, s, acc);
        if constexpr (kDot) {
            cpx<R> ww[12];
            load_spinor(static_cast<const SpT<R> *>(P.w), P.V, s, ww);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                z64 a = cast<double>(ww[k]), o = cast<double>(acc[k]);
                dr += a.r * o.r + a.i * o.i;
                di += a.r * o.i - a.i * o.r;
            }
        }
    }
    if constexpr (kDot) {
        __shared__ double lds[8];
        double v[2] = {dr, di};
        block_sum<2>(v, lds);
        if (threadIdx.x == 0) P.partials[blockIdx.x] = {v[0], v[1]};
    }
}

template <typename R, typename LT>
void launch_typed(const StencilParams &P, int nblk, bool epi, bool dot, hipStream_t s)
{
    dim3 g(nblk), b(256);
    if (dot)
        hipLaunchKernelGGL((stencil_kernel<R, LT, true, true>), g, b, 0, s, P);
    else if (epi)
        hipLaunchKernelGGL((stencil_kernel<R, LT, true, false>), g, b, 0, s, P);
    else
        hipLaunchKernelGGL((stencil_kernel<R, LT, false, false>), g, b, 0, s, P);
}

}  // namespace

int dslash_blocks(const Lattice &lat) { return (int)((lat.V + 255) / 256); }

int dslash_launch(const Lattice &lat, sgn_prec p, const OpSpec &op, const void *in, void *out,
                  const Epilogue &ep, hipStream_t s)
{
    StencilParams P{};
    P.in = in;
    P.out = out;
    P.V = (int)lat.V;
    for (int d = 0; d < 4; ++d) {
        P.L[d] = lat.L[d];
        P.bcf[d] = (float)lat.bc[d];
    }
    P.stride[0] = 1;
    P.stride[1] = lat.L[0];
    P.stride[2] = lat.L[0] * lat.L[1];
    P.stride[3] = lat.L[0] * lat.L[1] * lat.L[2];
    P.kappa = lat.kappa;
    P.wf_t = std::exp(-op.mu);
    P.wb_t = std::exp(op.mu);
    P.s5_in = op.g5_in ? -1.f : 1.f;
    P.s5_out = op.g5_out ? -1.f : 1.f;
    P.a = ep.a;
    P.b = ep.b;
    P.b_dev = ep.b_dev;
    P.z = ep.z;
    P.w = ep.w;
    P.partials = ep.partials;
    P.in_scale = ep.in_scale;
    const bool dot = ep.w != nullptr;
    const bool epi = dot || ep.z != nullptr || ep.a != 1.0 || ep.in_scale != nullptr;
    if (dot && !ep.partials) throw Failure{SGN_ERR_INVALID, "stencil dot without partial buffer"};
    const int nblk = dslash_blocks(lat);
    // algorithmic bytes: in and out spinors once, the 4 links of each site once,
    // plus the epilogue operands; 1368 flop per site for the stencil itself
    const double sb = (p == SGN_PREC_F64) ? 192.0 : 96.0;
    const double lb = (p == SGN_PREC_F64) ? 144.0 : (p == SGN_PREC_F32 ? 72.0 : 36.0);
    const double site_bytes = 2 * sb + 4 * lb + (ep.z ? sb : 0.0) + (dot ? sb : 0.0);
    const double site_flops = 1368.0 + (epi ? 24.0 : 0.0) + (ep.z ? 96.0 : 0.0) + (dot ? 96.0 : 0.0);
    const int prof = lat.ctx->prof_start(s);
    switch (p) {
    case SGN_PREC_F64:
        if (!lat.links64) throw Failure{SGN_ERR_INVALID, "lattice has no FP64 links"};
        P.links = lat.links64;
        launch_typed<double, double2>(P, nblk, epi, dot, s);
        break;
    case SGN_PREC_F32:
        if (!lat.links32) throw Failure{SGN_ERR_INVALID, "lattice has no FP32 links"};
        P.links = lat.links32;
        launch_typed<float, float2>(P, nblk, epi, dot, s);
        break;
    case SGN_PREC_F32_H16:
        if (!lat.links16) throw Failure{SGN_ERR_INVALID, "lattice has no FP16 links"};
        P.links = lat.links16;
        launch_typed<float, __half2>(P, nblk, epi, dot, s);
        break;
    default:
        throw Failure{SGN_ERR_INVALID, "unknown precision"};
    }
    SGN_HIP(hipGetLastError());
    lat.ctx->prof_stop(prof, s, p == SGN_PREC_F64 ? SGN_K_STENCIL_F64 : (p == SGN_PREC_F32 ? SGN_K_STENCIL_F32 : SGN_K_STENCIL_H16),
                       site_bytes * lat.V, site_flops * lat.V);
    return nblk;
}

}  // namespace sgn

// ----------------------------------------------------------------------------- C ABI
using namespace sgn;

static sgn_status apply_common(sgn_lattice l, double mu, const void *in, void *out, sgn_prec p,
                               unsigned flags, void *stream, bool dag)
{
    return guard([&] {
        SGN_REQUIRE(l != nullptr && in != nullptr && out != nullptr, "wilson_apply: null argument");
        SGN_REQUIRE(in != out, "wilson_apply: in and out must differ");
        SGN_REQUIRE(std::isfinite(mu), "wilson_apply: mu is not finite");
        Lattice &lat = *as_lattice(l);
        SGN_HIP(hipSetDevice(lat.ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        OpSpec op;
        const bool g5 = !(flags & SGN_NO_GAMMA5);
        if (!dag) {
            op.mu = mu;
            op.g5_out = g5;
            op.g5_in = false;
        } else if (g5) {   // H(mu)^H = H(-mu)
            op.mu = -mu;
            op.g5_out = true;
            op.g5_in = false;
        } else {           // D(mu)^H = gamma5 D(-mu) gamma5
            op.mu = -mu;
            op.g5_out = true;
            op.g5_in = true;
        }
        Epilogue ep;
        if (flags & SGN_INTERNAL_LAYOUT) {
            dslash_launch(lat, p, op, in, out, ep, s);
        } else {
            const size_t bytes = spinor_bytes(lat.V, p);
            lat.ensure_stage(bytes);
            pack_spinor(lat, in, lat.stage_in, p, s);
            dslash_launch(lat, p, op, lat.stage_in, lat.stage_out, ep, s);
            unpack_spinor(lat, lat.stage_out, out, p, s);
        }
    });
}

extern "C" sgn_status wilson_apply(sgn_lattice lat, double mu, const void *in, void *out, sgn_prec p,
                                   unsigned flags, void *stream)
{
    return apply_common(lat, mu, in, out, p, flags, stream, false);
}

extern "C" sgn_status wilson_apply_dag(sgn_lattice lat, double mu, const void *in, void *out, sgn_prec p,
                                       unsigned flags, void *stream)
{
    return apply_common(lat, mu, in, out, p, flags, stream, true);
}
