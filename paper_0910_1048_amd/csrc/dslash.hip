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
#ifndef SGN_STENCIL_THREADS
#define SGN_STENCIL_THREADS 256
#endif
#ifndef SGN_XCD_REMAP
#define SGN_XCD_REMAP 1
#endif
#ifndef SGN_T_MINOR
#define SGN_T_MINOR 1   // t-fastest block order inside each XCD's t-slab when the shape allows
#endif
#ifndef SGN_STENCIL_LDS_PAD
#define SGN_STENCIL_LDS_PAD 0
#endif
#ifndef SGN_PIN_PAIR
#define SGN_PIN_PAIR 0   // 1: both hops of a direction in flight together
#endif
#ifndef SGN_STENCIL_LDS
#define SGN_STENCIL_LDS 1   // single-RHS stencil with the block's own spinors staged in LDS
#endif
#ifndef SGN_STAGED_STRIP
#define SGN_STAGED_STRIP 1   // staged kernel block order: 0 = z-fastest XCD t-slabs, W > 0 = t-fastest strips of W blocks
#endif
#ifndef SGN_LDS_MAXBYTES
#define SGN_LDS_MAXBYTES 64512   // dynamic LDS budget of one block of the staged stencil (64 KiB less the reduction scratch)
#endif

namespace sgn {

namespace {

}  // namespace
constexpr int kMaxRhs = 2;
namespace {

struct RhsParams {
    const void *in;
    void *out;
    double wf_t, wb_t;  // time-hop weights e^{-mu}, e^{+mu} of this right-hand side
    float s5_in;        // -1: apply gamma5 to the input first
    float s5_out;       // -1: apply gamma5 to the result
    // epilogue  out = a * in_scale * Op(in) + b * z ;  partials of conj(w) . out
    double a;
    z64 b;
    const z64 *b_dev;
    const void *z;
    const void *w;
    z64 *partials;
    const z64 *in_scale;
    int norm;  // with w: partials hold {conj(w) . out, ||out||^2} per block
};

struct StencilParams {
    const void *links;
    int V;  // sites
    int S;  // component stride
    int L[4];
    int stride[4];
    float bcf[4];  // boundary factor per direction (hops that wrap)
    double kappa;
    // block schedule: when sched_T > 0, XCD k owns the t-slab [k*T, (k+1)*T) and
    // walks it region by region with t fastest (sched_R spatial regions per slice)
    int sched_T, sched_R;
    int nblk_sites;  // blocks covering the V sites; later blocks zero the padding sites [V, S)
    int blk_sites;   // staged kernel: sites per block (whole x-rows)
    int nblk_total;  // blocks of this application (sites + padding); batched launches skip the rest
    int link_ne;     // complex entries stored per link (6 or 9)
    RhsParams rhs[kMaxRhs];
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

template <int NU, int NR, typename R, typename LT>
__device__ __forceinline__ void hop_pair(cpx<R> (&acc)[NR][12], const StencilParams &P, int s, int coord)
{
    const LT *U = static_cast<const LT *>(P.links);
    const int L = P.L[NU], st = P.stride[NU];
    const R kap = static_cast<R>(P.kappa);
    cpx<R> u[9];
    // forward hop: (1 - gamma) U_nu(x) psi(x + nu), the link shared by all right-hand sides
    {
        const bool wrap = coord == L - 1;
        const int n = wrap ? s - (L - 1) * st : s + st;
        const R bcf = wrap ? static_cast<R>(P.bcf[NU]) : R(1);
        load_link<R>(U, P.S, P.link_ne, NU, s, u);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cpx<R> p[12], h[6], chi[6];
            load_spinor(static_cast<const SpT<R> *>(P.rhs[r].in), P.S, n, p);
            const R s5 = static_cast<R>(P.rhs[r].s5_in);
#pragma unroll
            for (int k = 6; k < 12; ++k) p[k] = s5 * p[k];
            project<NU, true>(p, h);
            link_mul<false>(u, h, chi);
            const R w = NU == 3 ? static_cast<R>(P.rhs[r].wf_t) : R(1);
            accumulate<NU, true>(acc[r], chi, -kap * w * bcf);
        }
    }
    if (!SGN_PIN_PAIR) {
#pragma unroll
        for (int r = 0; r < NR; ++r) pin(acc[r]);
    }
    // backward hop: (1 + gamma) U_nu(x - nu)^H psi(x - nu)
    {
        const bool wrap = coord == 0;
        const int n = wrap ? s + (L - 1) * st : s - st;
        const R bcb = wrap ? static_cast<R>(P.bcf[NU]) : R(1);
        load_link<R>(U, P.S, P.link_ne, NU, n, u);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cpx<R> p[12], h[6], chi[6];
            load_spinor(static_cast<const SpT<R> *>(P.rhs[r].in), P.S, n, p);
            const R s5 = static_cast<R>(P.rhs[r].s5_in);
#pragma unroll
            for (int k = 6; k < 12; ++k) p[k] = s5 * p[k];
            project<NU, false>(p, h);
            link_mul<true>(u, h, chi);
            const R w = NU == 3 ? static_cast<R>(P.rhs[r].wb_t) : R(1);
            accumulate<NU, false>(acc[r], chi, -kap * w * bcb);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) pin(acc[r]);
}

template <typename R, typename LT, int NR, bool kEpi, bool kDot>
__global__ void __launch_bounds__(SGN_STENCIL_THREADS) __attribute__((amdgpu_waves_per_eu(SGN_STENCIL_WAVES))) stencil_kernel(StencilParams P)
{
    if ((int)blockIdx.x >= P.nblk_sites) {  // padding of the component arrays: keep it zero
        const int s = P.V + ((int)blockIdx.x - P.nblk_sites) * SGN_STENCIL_THREADS + threadIdx.x;
        if (s < P.S) {
            cpx<R> zero[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) zero[k] = {R(0), R(0)};
#pragma unroll
            for (int r = 0; r < NR; ++r) store_spinor(static_cast<SpT<R> *>(P.rhs[r].out), P.S, s, zero);
        }
        if constexpr (kDot) {
            if (threadIdx.x == 0)
                for (int r = 0; r < NR; ++r)
                    if (P.rhs[r].w) {
                        if (P.rhs[r].norm) {
                            P.rhs[r].partials[2 * blockIdx.x] = {0.0, 0.0};
                            P.rhs[r].partials[2 * blockIdx.x + 1] = {0.0, 0.0};
                        } else {
                            P.rhs[r].partials[blockIdx.x] = {0.0, 0.0};
                        }
                    }
        }
        return;
    }
    int blk;
    if (P.sched_T > 0) {
        // t-minor order inside each XCD's slab: the t-neighbours of a block are the
        // blocks just before and after it
        const int k = blockIdx.x % 8, j = blockIdx.x / 8;
        const int tl = j % P.sched_T, r = j / P.sched_T;
        blk = (k * P.sched_T + tl) * P.sched_R + r;
    } else {
        blk = SGN_XCD_REMAP ? xcd_block(blockIdx.x, P.nblk_sites) : (int)blockIdx.x;
    }
    const int s = blk * SGN_STENCIL_THREADS + threadIdx.x;
    const bool valid = s < P.V;
    double dr[NR], di[NR], dn[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dr[r] = di[r] = dn[r] = 0.0;
    if (valid) {
        int c0 = s % P.L[0];
        int q = s / P.L[0];
        int c1 = q % P.L[1];
        q /= P.L[1];
        int c2 = q % P.L[2];
        int c3 = q / P.L[2];
        cpx<R> acc[NR][12];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            load_spinor(static_cast<const SpT<R> *>(P.rhs[r].in), P.S, s, acc[r]);
            const R s5 = static_cast<R>(P.rhs[r].s5_in);
#pragma unroll
            for (int k = 6; k < 12; ++k) acc[r][k] = s5 * acc[r][k];
        }
        hop_pair<0, NR, R, LT>(acc, P, s, c0);
        hop_pair<1, NR, R, LT>(acc, P, s, c1);
        hop_pair<2, NR, R, LT>(acc, P, s, c2);
        hop_pair<3, NR, R, LT>(acc, P, s, c3);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const RhsParams &Q = P.rhs[r];
            const R s5o = static_cast<R>(Q.s5_out);
#pragma unroll
            for (int k = 6; k < 12; ++k) acc[r][k] = s5o * acc[r][k];
            if constexpr (kEpi) {
                cpx<R> sc = {static_cast<R>(Q.a), R(0)};
                if (Q.in_scale) {
                    z64 t = *Q.in_scale;
                    sc = {static_cast<R>(Q.a * t.r), static_cast<R>(Q.a * t.i)};
                }
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[r][k] = sc * acc[r][k];
                if (Q.z) {
                    z64 bb = Q.b;
                    if (Q.b_dev) {
                        z64 t = *Q.b_dev;
                        bb = {bb.r * t.r - bb.i * t.i, bb.r * t.i + bb.i * t.r};
                    }
                    cpx<R> b = {static_cast<R>(bb.r), static_cast<R>(bb.i)};
                    cpx<R> zz[12];
                    load_spinor(static_cast<const SpT<R> *>(Q.z), P.S, s, zz);
#pragma unroll
                    for (int k = 0; k < 12; ++k) acc[r][k] = acc[r][k] + b * zz[k];
                }
            }
            store_spinor(static_cast<SpT<R> *>(Q.out), P.S, s, acc[r]);
            if constexpr (kDot) {
                if (Q.w) {
                    cpx<R> ww[12];
                    load_spinor(static_cast<const SpT<R> *>(Q.w), P.S, s, ww);
#pragma unroll
                    for (int k = 0; k < 12; ++k) {
                        z64 a = cast<double>(ww[k]), o = cast<double>(acc[r][k]);
                        dr[r] += a.r * o.r + a.i * o.i;
                        di[r] += a.r * o.i - a.i * o.r;
                        dn[r] += o.r * o.r + o.i * o.i;
                    }
                }
            }
        }
    }
    if constexpr (kDot) {
        __shared__ double lds[3 * (SGN_STENCIL_THREADS / 64)];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!P.rhs[r].w) continue;  // uniform
            double v[3] = {dr[r], di[r], dn[r]};
            block_sum<3>(v, lds);
            if (threadIdx.x == 0) {
                if (P.rhs[r].norm) {
                    P.rhs[r].partials[2 * blockIdx.x] = {v[0], v[1]};
                    P.rhs[r].partials[2 * blockIdx.x + 1] = {v[2], 0.0};
                } else {
                    P.rhs[r].partials[blockIdx.x] = {v[0], v[1]};
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------- staged stencil
// Single right-hand side.  A block owns B consecutive sites made of whole
// x-rows (whole x-y planes when they fit), so the +-x neighbours of every site
// and, for whole planes, the +-y neighbours too lie inside the block.  Each
// thread loads its own spinor once (it is needed for the diagonal term anyway)
// and stores it in LDS; a neighbour inside the block is then read from LDS and
// only the others (+-z, +-t, block-edge rows) are gathered from memory.

// largest block of the staged kernel: FP64 needs ~160 VGPRs, so at most 2 waves per SIMD
template <typename R> constexpr int kStagedMaxThreads = sizeof(R) == 8 ? 512 : 1024;

template <typename R>
__device__ __forceinline__ void lds_store_spinor(SpT<R> *l, int B, int i, const cpx<R> v[12]);
template <>
__device__ __forceinline__ void lds_store_spinor<double>(double2 *l, int B, int i, const cpx<double> v[12])
{
#pragma unroll
    for (int c = 0; c < 12; ++c) l[c * B + i] = make_double2(v[c].r, v[c].i);
}
template <>
__device__ __forceinline__ void lds_store_spinor<float>(float4 *l, int B, int i, const cpx<float> v[12])
{
#pragma unroll
    for (int c = 0; c < 6; ++c) l[c * B + i] = make_float4(v[2 * c].r, v[2 * c].i, v[2 * c + 1].r, v[2 * c + 1].i);
}

template <typename R>
__device__ __forceinline__ void lds_load_spinor(const SpT<R> *l, int B, int i, cpx<R> v[12]);
template <>
__device__ __forceinline__ void lds_load_spinor<double>(const double2 *l, int B, int i, cpx<double> v[12])
{
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 t = l[c * B + i];
        v[c] = {t.x, t.y};
    }
}
template <>
__device__ __forceinline__ void lds_load_spinor<float>(const float4 *l, int B, int i, cpx<float> v[12])
{
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        float4 t = l[c * B + i];
        v[2 * c] = {t.x, t.y};
        v[2 * c + 1] = {t.z, t.w};
    }
}

// neighbour spinor n: from LDS when it belongs to this block (stored already
// multiplied by the input gamma5 sign), else from memory
template <typename R>
__device__ __forceinline__ void fetch_neighbour(const StencilParams &P, const SpT<R> *lds, int base, int n,
                                                cpx<R> p[12])
{
    const int ln = n - base;
    if ((unsigned)ln < (unsigned)P.blk_sites) {
        lds_load_spinor<R>(lds, P.blk_sites, ln, p);
    } else {
        load_spinor(static_cast<const SpT<R> *>(P.rhs[0].in), P.S, n, p);
        const R s5 = static_cast<R>(P.rhs[0].s5_in);
#pragma unroll
        for (int k = 6; k < 12; ++k) p[k] = s5 * p[k];
    }
}

template <int NU, typename R, typename LT>
__device__ __forceinline__ void hop_pair_staged(cpx<R> (&acc)[12], const StencilParams &P, const SpT<R> *lds,
                                                int base, int s, int coord)
{
    const LT *U = static_cast<const LT *>(P.links);
    const int L = P.L[NU], st = P.stride[NU];
    const R kap = static_cast<R>(P.kappa);
    cpx<R> u[9];
    {
        const bool wrap = coord == L - 1;
        const int n = wrap ? s - (L - 1) * st : s + st;
        const R bcf = wrap ? static_cast<R>(P.bcf[NU]) : R(1);
        cpx<R> p[12], h[6], chi[6];
        load_link<R>(U, P.S, P.link_ne, NU, s, u);
        fetch_neighbour<R>(P, lds, base, n, p);
        project<NU, true>(p, h);
        link_mul<false>(u, h, chi);
        const R w = NU == 3 ? static_cast<R>(P.rhs[0].wf_t) : R(1);
        accumulate<NU, true>(acc, chi, -kap * w * bcf);
    }
    pin(acc);
    {
        const bool wrap = coord == 0;
        const int n = wrap ? s + (L - 1) * st : s - st;
        const R bcb = wrap ? static_cast<R>(P.bcf[NU]) : R(1);
        cpx<R> p[12], h[6], chi[6];
        load_link<R>(U, P.S, P.link_ne, NU, n, u);
        fetch_neighbour<R>(P, lds, base, n, p);
        project<NU, false>(p, h);
        link_mul<true>(u, h, chi);
        const R w = NU == 3 ? static_cast<R>(P.rhs[0].wb_t) : R(1);
        accumulate<NU, false>(acc, chi, -kap * w * bcb);
    }
    pin(acc);
}

template <typename R, typename LT, bool kEpi, bool kDot>
__device__ __forceinline__ void staged_body(const StencilParams &P, const int bx)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SpT<R> *lds = reinterpret_cast<SpT<R> *>(smem_raw);
    const RhsParams &Q = P.rhs[0];
    if (bx >= P.nblk_sites) {  // padding of the component arrays: keep it zero
        const int s = P.V + (bx - P.nblk_sites) * (int)blockDim.x + (int)threadIdx.x;
        if (s < P.S) {
            cpx<R> zero[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) zero[k] = {R(0), R(0)};
            store_spinor(static_cast<SpT<R> *>(Q.out), P.S, s, zero);
        }
        if constexpr (kDot) {
            if (threadIdx.x == 0 && Q.w) {
                if (Q.norm) {
                    Q.partials[2 * bx] = {0.0, 0.0};
                    Q.partials[2 * bx + 1] = {0.0, 0.0};
                } else {
                    Q.partials[bx] = {0.0, 0.0};
                }
            }
        }
        return;
    }
    const int B = P.blk_sites;
    int blk;
    if (P.sched_T > 0) {
        // XCD k owns the t-slab [k T, (k+1) T) of sched_R blocks per t-slice and
        // walks it in strips of W consecutive blocks with t fastest, so the
        // t-neighbours of a block run on the same XCD at about the same time
        const int W = SGN_STAGED_STRIP;
        const int k = bx % 8, j = bx / 8;
        const int per_strip = P.sched_T * W;
        const int strip = j / per_strip, rem = j - strip * per_strip;
        const int tl = rem / W, wi = rem - tl * W;
        blk = (k * P.sched_T + tl) * P.sched_R + strip * W + wi;
    } else {
        blk = SGN_XCD_REMAP ? xcd_block(bx, P.nblk_sites) : bx;
    }
    const int base = blk * B;
    const int i = threadIdx.x;
    const int s = base + i;
    const bool valid = i < B;  // blocks tile the V sites exactly
    cpx<R> acc[12];
    if (valid) {
        load_spinor(static_cast<const SpT<R> *>(Q.in), P.S, s, acc);
        const R s5 = static_cast<R>(Q.s5_in);
#pragma unroll
        for (int k = 6; k < 12; ++k) acc[k] = s5 * acc[k];
        lds_store_spinor<R>(lds, B, i, acc);
    }
    __syncthreads();
    double dr = 0.0, di = 0.0, dn = 0.0;
    if (valid) {
        int c0 = s % P.L[0];
        int q = s / P.L[0];
        int c1 = q % P.L[1];
        q /= P.L[1];
        int c2 = q % P.L[2];
        int c3 = q / P.L[2];
        hop_pair_staged<0, R, LT>(acc, P, lds, base, s, c0);
        hop_pair_staged<1, R, LT>(acc, P, lds, base, s, c1);
        hop_pair_staged<2, R, LT>(acc, P, lds, base, s, c2);
        hop_pair_staged<3, R, LT>(acc, P, lds, base, s, c3);
        const R s5o = static_cast<R>(Q.s5_out);
#pragma unroll
        for (int k = 6; k < 12; ++k) acc[k] = s5o * acc[k];
        if constexpr (kEpi) {
            cpx<R> sc = {static_cast<R>(Q.a), R(0)};
            if (Q.in_scale) {
                z64 t = *Q.in_scale;
                sc = {static_cast<R>(Q.a * t.r), static_cast<R>(Q.a * t.i)};
            }
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = sc * acc[k];
            if (Q.z) {
                z64 bb = Q.b;
                if (Q.b_dev) {
                    z64 t = *Q.b_dev;
                    bb = {bb.r * t.r - bb.i * t.i, bb.r * t.i + bb.i * t.r};
                }
                cpx<R> b = {static_cast<R>(bb.r), static_cast<R>(bb.i)};
                cpx<R> zz[12];
                load_spinor(static_cast<const SpT<R> *>(Q.z), P.S, s, zz);
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = acc[k] + b * zz[k];
            }
        }
        store_spinor(static_cast<SpT<R> *>(Q.out), P.S, s, acc);
        if constexpr (kDot) {
            if (Q.w) {
                cpx<R> ww[12];
                load_spinor(static_cast<const SpT<R> *>(Q.w), P.S, s, ww);
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    z64 a = cast<double>(ww[k]), o = cast<double>(acc[k]);
                    dr += a.r * o.r + a.i * o.i;
                    di += a.r * o.i - a.i * o.r;
                    dn += o.r * o.r + o.i * o.i;
                }
            }
        }
    }
    if constexpr (kDot) {
        __shared__ double red[3 * 16];
        if (Q.w) {  // uniform
            double v[3] = {dr, di, dn};
            block_sum<3>(v, red);
            if (threadIdx.x == 0) {
                if (Q.norm) {
                    Q.partials[2 * bx] = {v[0], v[1]};
                    Q.partials[2 * bx + 1] = {v[2], 0.0};
                } else {
                    Q.partials[bx] = {v[0], v[1]};
                }
            }
        }
    }
}

template <typename R, typename LT, bool kEpi, bool kDot>
__global__ void __launch_bounds__(kStagedMaxThreads<R>) stencil_staged_kernel(StencilParams P)
{
    staged_body<R, LT, kEpi, kDot>(P, (int)blockIdx.x);
}

// Batched form: blockIdx.y selects one of several independent applications
// (own lattice, fields and epilogue) whose parameters live in device memory.
// gridDim.x is a multiple of 8, so the XCD of block (x, y) is x mod 8 as in
// the single form.
template <typename R, typename LT, bool kEpi, bool kDot>
__global__ void __launch_bounds__(kStagedMaxThreads<R>) stencil_staged_batch(const StencilParams *__restrict__ plist)
{
    const StencilParams P = plist[blockIdx.y];
    if ((int)blockIdx.x >= P.nblk_total) return;
    staged_body<R, LT, kEpi, kDot>(P, (int)blockIdx.x);
}

template <typename R, typename LT>
void launch_staged(const StencilParams &P, int nblk, int threads, size_t lds, bool epi, bool dot, hipStream_t s)
{
    dim3 g(nblk), b(threads);
    if (dot)
        hipLaunchKernelGGL((stencil_staged_kernel<R, LT, true, true>), g, b, lds, s, P);
    else if (epi)
        hipLaunchKernelGGL((stencil_staged_kernel<R, LT, true, false>), g, b, lds, s, P);
    else
        hipLaunchKernelGGL((stencil_staged_kernel<R, LT, false, false>), g, b, lds, s, P);
}

template <typename R, typename LT, int NR>
void launch_typed(const StencilParams &P, int nblk, bool epi, bool dot, hipStream_t s)
{
    dim3 g(nblk), b(SGN_STENCIL_THREADS);
    if (dot)
        hipLaunchKernelGGL((stencil_kernel<R, LT, NR, true, true>), g, b, 0, s, P);
    else if (epi)
        hipLaunchKernelGGL((stencil_kernel<R, LT, NR, true, false>), g, b, 0, s, P);
    else
        hipLaunchKernelGGL((stencil_kernel<R, LT, NR, false, false>), g, b, 0, s, P);
}

template <typename R, typename LT>
void launch_nr(const StencilParams &P, int nr, int nblk, bool epi, bool dot, hipStream_t s)
{
    switch (nr) {
    case 1: launch_typed<R, LT, 1>(P, nblk, epi, dot, s); break;
    case 2: launch_typed<R, LT, 2>(P, nblk, epi, dot, s); break;
    default: throw Failure{SGN_ERR_INVALID, "stencil: unsupported number of right-hand sides"};
    }
}

}  // namespace

namespace {

// Block shape of the staged kernel: B sites of whole x-rows (whole x-y planes
// when they fit the LDS budget), B dividing V; not used when B < 64.
struct StagedPlan {
    bool ok = false;
    int B = 0, threads = 0, nblk_sites = 0, nblk = 0;
    size_t lds = 0;
};

StagedPlan staged_plan(const Lattice &lat, sgn_prec p)
{
    StagedPlan pl;
    if (!SGN_STENCIL_LDS) return pl;
    const int64_t site_bytes = p == SGN_PREC_F64 ? 192 : 96;
    const int64_t bmax = std::min<int64_t>(p == SGN_PREC_F64 ? kStagedMaxThreads<double> : kStagedMaxThreads<float>,
                                           SGN_LDS_MAXBYTES / site_bytes);
    const int64_t Lx = lat.L[0], A = (int64_t)lat.L[0] * lat.L[1];
    const int64_t nplane = (int64_t)lat.L[2] * lat.L[3];
    int64_t B = 0;
    if (A <= bmax) {
        int64_t P = bmax / A;
        while (nplane % P) --P;
        B = P * A;
    } else {
        int64_t rows = bmax / Lx;
        const int64_t nrows = (int64_t)lat.L[1] * nplane;
        while (rows > 0 && nrows % rows) --rows;
        B = rows * Lx;
    }
    if (B < 64) return pl;
    pl.ok = true;
    pl.B = (int)B;
    pl.threads = (int)((B + 63) / 64 * 64);
    pl.nblk_sites = (int)(lat.V / B);
    const int64_t pad = lat.S > lat.V ? (lat.S - lat.V + pl.threads - 1) / pl.threads : 0;
    pl.nblk = pl.nblk_sites + (int)pad;
    pl.lds = (size_t)B * site_bytes;
    return pl;
}

}  // namespace

int dslash_blocks(const Lattice &lat)
{
    const int64_t t = SGN_STENCIL_THREADS;
    const int64_t valid = (lat.V + t - 1) / t;
    const int64_t pad = lat.S > lat.V ? (lat.S - lat.V + t - 1) / t : 0;  // padding sites [V, S)
    int n = (int)(valid + pad);
    for (sgn_prec p : {SGN_PREC_F64, SGN_PREC_F32}) {
        const StagedPlan pl = staged_plan(lat, p);
        if (pl.ok) n = std::max(n, pl.nblk);
    }
    return n;
}

namespace {

// Everything about one stencil application except the launch itself.
struct PreparedStencil {
    StencilParams P{};
    StagedPlan pl;
    int nblk = 0;       // blocks of the launch (= partials written when dotting)
    double bytes = 0.0;  // algorithmic bytes and flops
    double flops = 0.0;
    bool epi = false, dot = false;
};

PreparedStencil prepare_stencil(const Lattice &lat, sgn_prec p, int nr, const OpSpec *op, const void *const *in,
                                void *const *out, const Epilogue *ep)
{
    if (nr < 1 || nr > kMaxRhs) throw Failure{SGN_ERR_INVALID, "stencil: 1..2 right-hand sides per launch"};
    PreparedStencil ps;
    StencilParams &P = ps.P;
    P.V = (int)lat.V;
    P.S = (int)lat.S;
    for (int d = 0; d < 4; ++d) {
        P.L[d] = lat.L[d];
        P.bcf[d] = (float)lat.bc[d];
    }
    P.stride[0] = 1;
    P.stride[1] = lat.L[0];
    P.stride[2] = lat.L[0] * lat.L[1];
    P.stride[3] = lat.L[0] * lat.L[1] * lat.L[2];
    P.kappa = lat.kappa;
    double extra_bytes = 0.0, extra_flops = 0.0;
    const double sb = (p == SGN_PREC_F64) ? 192.0 : 96.0;
    for (int r = 0; r < nr; ++r) {
        RhsParams &Q = P.rhs[r];
        Q.in = in[r];
        Q.out = out[r];
        Q.wf_t = std::exp(-op[r].mu);
        Q.wb_t = std::exp(op[r].mu);
        Q.s5_in = op[r].g5_in ? -1.f : 1.f;
        Q.s5_out = op[r].g5_out ? -1.f : 1.f;
        Q.a = ep[r].a;
        Q.b = ep[r].b;
        Q.b_dev = ep[r].b_dev;
        Q.z = ep[r].z;
        Q.w = ep[r].w;
        Q.partials = ep[r].partials;
        Q.in_scale = ep[r].in_scale;
        Q.norm = ep[r].norm ? 1 : 0;
        if (ep[r].w && !ep[r].partials) throw Failure{SGN_ERR_INVALID, "stencil dot without partial buffer"};
        ps.dot = ps.dot || ep[r].w != nullptr;
        ps.epi = ps.epi || ep[r].w != nullptr || ep[r].z != nullptr || ep[r].a != 1.0 || ep[r].in_scale != nullptr;
        extra_bytes += (ep[r].z ? sb : 0.0) + (ep[r].w ? sb : 0.0);
        extra_flops += (ep[r].z ? 96.0 : 0.0) + (ep[r].w ? 96.0 : 0.0) + 24.0;
    }
    {
        const int64_t t = SGN_STENCIL_THREADS;
        ps.nblk = (int)((lat.V + t - 1) / t + (lat.S > lat.V ? (lat.S - lat.V + t - 1) / t : 0));
    }
    P.nblk_sites = (int)((lat.V + SGN_STENCIL_THREADS - 1) / SGN_STENCIL_THREADS);
    {
        const int64_t vxyz = (int64_t)lat.L[0] * lat.L[1] * lat.L[2];
        P.sched_T = P.sched_R = 0;
        if (SGN_T_MINOR && vxyz % SGN_STENCIL_THREADS == 0 && lat.L[3] % 8 == 0) {
            P.sched_T = lat.L[3] / 8;
            P.sched_R = (int)(vxyz / SGN_STENCIL_THREADS);
            if ((int64_t)8 * P.sched_T * P.sched_R != P.nblk_sites) P.sched_T = P.sched_R = 0;
        }
    }
    // algorithmic bytes: every input and output spinor once, the 4 links of each
    // site once (shared by the right-hand sides), plus the epilogue operands;
    // 1368 flop per site and right-hand side for the stencil itself
    P.link_ne = lat.link_ne;
    const double lb = lat.link_ne * ((p == SGN_PREC_F64) ? 16.0 : (p == SGN_PREC_F32 ? 8.0 : 4.0));
    ps.bytes = (2 * sb * nr + 4 * lb + extra_bytes) * lat.V;
    ps.flops = (1368.0 * nr + extra_flops) * lat.V;
    ps.pl = nr == 1 ? staged_plan(lat, p) : StagedPlan{};
    if (ps.pl.ok) {
        P.blk_sites = ps.pl.B;
        P.nblk_sites = ps.pl.nblk_sites;
        ps.nblk = ps.pl.nblk;
        P.sched_T = P.sched_R = 0;
        const int64_t v3 = (int64_t)lat.L[0] * lat.L[1] * lat.L[2];
        if (SGN_STAGED_STRIP > 0 && v3 % ps.pl.B == 0 && lat.L[3] % 8 == 0 && (v3 / ps.pl.B) % SGN_STAGED_STRIP == 0) {
            P.sched_T = lat.L[3] / 8;
            P.sched_R = (int)(v3 / ps.pl.B);
        }
    }
    P.nblk_total = ps.nblk;
    switch (p) {
    case SGN_PREC_F64: P.links = lat.links64; break;
    case SGN_PREC_F32: P.links = lat.links32; break;
    case SGN_PREC_F32_H16: P.links = lat.links16; break;
    default: throw Failure{SGN_ERR_INVALID, "unknown precision"};
    }
    if (!P.links)
        throw Failure{SGN_ERR_INVALID, p == SGN_PREC_F64 ? "lattice has no FP64 links"
                                                         : (p == SGN_PREC_F32 ? "lattice has no FP32 links"
                                                                              : "lattice has no FP16 links")};
    return ps;
}

int kclass(sgn_prec p)
{
    return p == SGN_PREC_F64 ? SGN_K_STENCIL_F64 : (p == SGN_PREC_F32 ? SGN_K_STENCIL_F32 : SGN_K_STENCIL_H16);
}

template <typename R, typename LT>
void launch_staged_batch(const StencilParams *dev, int count, int gx, int threads, size_t lds, bool epi, bool dot,
                         hipStream_t s)
{
    dim3 g(gx, count), b(threads);
    if (dot)
        hipLaunchKernelGGL((stencil_staged_batch<R, LT, true, true>), g, b, lds, s, dev);
    else if (epi)
        hipLaunchKernelGGL((stencil_staged_batch<R, LT, true, false>), g, b, lds, s, dev);
    else
        hipLaunchKernelGGL((stencil_staged_batch<R, LT, false, false>), g, b, lds, s, dev);
}

}  // namespace

int dslash_launch_multi(const Lattice &lat, sgn_prec p, int nr, const OpSpec *op, const void *const *in,
                        void *const *out, const Epilogue *ep, hipStream_t s)
{
    const PreparedStencil ps = prepare_stencil(lat, p, nr, op, in, out, ep);
    const int prof = lat.ctx->prof_start(s, kclass(p));
    switch (p) {
    case SGN_PREC_F64:
        if (ps.pl.ok)
            launch_staged<double, double2>(ps.P, ps.nblk, ps.pl.threads, ps.pl.lds, ps.epi, ps.dot, s);
        else
            launch_nr<double, double2>(ps.P, nr, ps.nblk, ps.epi, ps.dot, s);
        break;
    case SGN_PREC_F32:
        if (ps.pl.ok)
            launch_staged<float, float2>(ps.P, ps.nblk, ps.pl.threads, ps.pl.lds, ps.epi, ps.dot, s);
        else
            launch_nr<float, float2>(ps.P, nr, ps.nblk, ps.epi, ps.dot, s);
        break;
    default:
        if (ps.pl.ok)
            launch_staged<float, __half2>(ps.P, ps.nblk, ps.pl.threads, ps.pl.lds, ps.epi, ps.dot, s);
        else
            launch_nr<float, __half2>(ps.P, nr, ps.nblk, ps.epi, ps.dot, s);
        break;
    }
    SGN_HIP(hipGetLastError());
    lat.ctx->prof_stop(prof, s, kclass(p), ps.bytes, ps.flops);
    return ps.nblk;
}

StencilBatch::~StencilBatch()
{
    if (dev_) (void)hipFree(dev_);
}

void StencilBatch::prepare(const std::vector<StencilJob> &jobs, sgn_prec p)
{
    jobs_ = jobs;
    prec_ = p;
    nblk_.assign(jobs.size(), 0);
    batched_ = !jobs.empty();
    epi_ = dot_ = false;
    gx_ = threads_ = 0;
    lds_ = 0;
    bytes_ = flops_ = 0.0;
    std::vector<StencilParams> host(jobs.size());
    for (size_t k = 0; k < jobs.size(); ++k) {
        const StencilJob &j = jobs[k];
        const PreparedStencil ps = prepare_stencil(*j.lat, p, 1, &j.op, &j.in, &j.out, &j.ep);
        host[k] = ps.P;
        nblk_[k] = ps.nblk;
        batched_ = batched_ && ps.pl.ok;
        epi_ = epi_ || ps.epi;
        dot_ = dot_ || ps.dot;
        gx_ = std::max(gx_, ps.nblk);
        threads_ = std::max(threads_, ps.pl.threads);
        lds_ = std::max(lds_, ps.pl.lds);
        bytes_ += ps.bytes;
        flops_ += ps.flops;
    }
    gx_ = (gx_ + 7) / 8 * 8;
    if (!batched_) return;
    const size_t need = sizeof(StencilParams) * host.size();
    if (need > dev_bytes_) {
        if (dev_) SGN_HIP(hipFree(dev_));
        dev_ = nullptr;
        dev_bytes_ = 0;
        if (hipMalloc(&dev_, need) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "stencil batch parameters"};
        dev_bytes_ = need;
    }
    SGN_HIP(hipMemcpy(dev_, host.data(), need, hipMemcpyHostToDevice));
}

void StencilBatch::launch(hipStream_t s) const
{
    if (jobs_.empty()) return;
    if (!batched_) {  // some lattice has no staged block shape: one launch per application
        for (const StencilJob &j : jobs_) dslash_launch(*j.lat, prec_, j.op, j.in, j.out, j.ep, s);
        return;
    }
    Context *ctx = jobs_[0].lat->ctx;
    const int prof = ctx->prof_start(s, kclass(prec_));
    const StencilParams *d = static_cast<const StencilParams *>(dev_);
    const int cnt = (int)jobs_.size();
    switch (prec_) {
    case SGN_PREC_F64: launch_staged_batch<double, double2>(d, cnt, gx_, threads_, lds_, epi_, dot_, s); break;
    case SGN_PREC_F32: launch_staged_batch<float, float2>(d, cnt, gx_, threads_, lds_, epi_, dot_, s); break;
    default: launch_staged_batch<float, __half2>(d, cnt, gx_, threads_, lds_, epi_, dot_, s); break;
    }
    SGN_HIP(hipGetLastError());
    ctx->prof_stop(prof, s, kclass(prec_), bytes_, flops_);
}

int dslash_launch(const Lattice &lat, sgn_prec p, const OpSpec &op, const void *in, void *out,
                  const Epilogue &ep, hipStream_t s)
{
    return dslash_launch_multi(lat, p, 1, &op, &in, &out, &ep, s);
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
            const size_t bytes = spinor_bytes(lat.S, p);
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

extern "C" sgn_status wilson_apply_multi(sgn_lattice l, int nrhs, const double *mu, const void *const *in,
                                         void *const *out, sgn_prec p, unsigned flags, void *stream)
{
    return guard([&] {
        SGN_REQUIRE(l != nullptr && mu != nullptr && in != nullptr && out != nullptr && nrhs >= 0,
                    "wilson_apply_multi: null argument");
        SGN_REQUIRE(flags & SGN_INTERNAL_LAYOUT, "wilson_apply_multi: fields must be in the internal layout");
        Lattice &lat = *as_lattice(l);
        SGN_HIP(hipSetDevice(lat.ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        for (int i = 0; i < nrhs; ++i) {
            SGN_REQUIRE(in[i] && out[i] && std::isfinite(mu[i]), "wilson_apply_multi: bad right-hand side");
            for (int j = 0; j < nrhs; ++j)
                SGN_REQUIRE(in[i] != out[j], "wilson_apply_multi: inputs and outputs must not alias");
        }
        for (int i0 = 0; i0 < nrhs; i0 += kMaxRhs) {
            const int nr = std::min(kMaxRhs, nrhs - i0);
            OpSpec op[kMaxRhs];
            Epilogue ep[kMaxRhs];
            for (int r = 0; r < nr; ++r) {
                op[r].mu = mu[i0 + r];
                op[r].g5_out = !(flags & SGN_NO_GAMMA5);
            }
            dslash_launch_multi(lat, p, nr, op, in + i0, out + i0, ep, s);
        }
    });
}
