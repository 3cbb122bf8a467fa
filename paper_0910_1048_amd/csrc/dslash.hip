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
#include "launch.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>

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
#ifndef SGN_PIN_PAIR
#define SGN_PIN_PAIR 0   // 1: both hops of a direction in flight together
#endif
#ifndef SGN_STENCIL_LDS
#define SGN_STENCIL_LDS 1   // single-RHS stencil with the block's own spinors staged in LDS
#endif
#ifndef SGN_STAGED_STRIP
#define SGN_STAGED_STRIP 1   // staged kernel block order: 0 = z-fastest XCD t-slabs, W > 0 = t-fastest strips of W blocks
#endif
#ifndef SGN_NT_OUT
#define SGN_NT_OUT 1     // non-temporal stores of the stencil output
#endif
#ifndef SGN_LDS_MAXBYTES
#define SGN_LDS_MAXBYTES 64512   // dynamic LDS budget of one block of the staged stencil (64 KiB less the reduction scratch)
#endif

namespace sgn {

namespace {

}  // namespace
// right-hand sides of one multi-RHS application (one block walks all of them; a
// StencilParams holding this many is 2 KiB, within the kernel-argument limit)
constexpr int kMaxRhs = 16;
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
    int blk_sites;   // staged kernel: sites per block and t-slice (whole x-rows)
    int tslices;     // staged kernel: t-slices per block (1, or 2: a brick of the same B sites at t and t + 1)
    int nblk_total;  // blocks of this application (sites + padding); batched launches skip the rest
    int link_ne;     // complex entries stored per link (6 or 9)
    int tgauge;      // temporal gauge: U_t = 1 off the last time slice (the staged kernel skips those links)
    int nrhs;        // right-hand sides of this application (staged kernel; the unstaged one uses NR)
    RhsParams rhs[kMaxRhs];
};

// Complex arithmetic of the hops written as fused multiply-adds: a complex
// multiply-accumulate is four FMAs (the plain expression s + a * b compiles to
// two multiplies, two FMAs and two adds, as the compiler may not reassociate).

// s = a b, or s = conj(a) b with CONJ
template <bool CONJ, typename R>
__device__ __forceinline__ cpx<R> cmul_f(cpx<R> a, cpx<R> b)
{
    cpx<R> s;
    s.r = a.r * b.r;
    s.r = fma(CONJ ? a.i : -a.i, b.i, s.r);
    s.i = a.r * b.i;
    s.i = fma(CONJ ? -a.i : a.i, b.r, s.i);
    return s;
}

// s += a b, or s += conj(a) b with CONJ
template <bool CONJ, typename R>
__device__ __forceinline__ void cmac_f(cpx<R> &s, cpx<R> a, cpx<R> b)
{
    s.r = fma(a.r, b.r, s.r);
    s.r = fma(CONJ ? a.i : -a.i, b.i, s.r);
    s.i = fma(a.r, b.i, s.i);
    s.i = fma(CONJ ? -a.i : a.i, b.r, s.i);
}

// a + f * (ph b) for the phase ph in {+1, -1, +i, -i} (PH = 0, 1, 2, 3) and a real f
template <int PH, typename R>
__device__ __forceinline__ cpx<R> add_ph(cpx<R> a, R f, cpx<R> b)
{
    if constexpr (PH == 0) return {fma(f, b.r, a.r), fma(f, b.i, a.i)};
    else if constexpr (PH == 1) return {fma(-f, b.r, a.r), fma(-f, b.i, a.i)};
    else if constexpr (PH == 2) return {fma(-f, b.i, a.r), fma(f, b.r, a.i)};
    else return {fma(f, b.i, a.r), fma(-f, b.r, a.i)};
}

constexpr int kP1 = 0, kM1 = 1, kPI = 2, kMI = 3;

// Half-spinor projection (1 - gamma_nu) for FWD, (1 + gamma_nu) otherwise, of
// the spinor p with its lower two spins multiplied by s5 (the input gamma5
// sign, folded into the adds): h[0..2] = colour vector of the upper-spin-0
// row, h[3..5] = spin-1 row.
template <int NU, bool FWD, typename R>
__device__ __forceinline__ void project(const cpx<R> p[12], cpx<R> h[6], R s5)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cpx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if constexpr (NU == 0) {
            h[c] = FWD ? add_ph<kMI>(p0, s5, p3) : add_ph<kPI>(p0, s5, p3);
            h[3 + c] = FWD ? add_ph<kMI>(p1, s5, p2) : add_ph<kPI>(p1, s5, p2);
        } else if constexpr (NU == 1) {
            h[c] = FWD ? add_ph<kP1>(p0, s5, p3) : add_ph<kM1>(p0, s5, p3);
            h[3 + c] = FWD ? add_ph<kM1>(p1, s5, p2) : add_ph<kP1>(p1, s5, p2);
        } else if constexpr (NU == 2) {
            h[c] = FWD ? add_ph<kMI>(p0, s5, p2) : add_ph<kPI>(p0, s5, p2);
            h[3 + c] = FWD ? add_ph<kPI>(p1, s5, p3) : add_ph<kMI>(p1, s5, p3);
        } else {
            h[c] = FWD ? add_ph<kM1>(p0, s5, p2) : add_ph<kP1>(p0, s5, p2);
            h[3 + c] = FWD ? add_ph<kM1>(p1, s5, p3) : add_ph<kP1>(p1, s5, p3);
        }
    }
}

// acc += coef * reconstruct(chi): upper spins are chi0, chi1; lower spins follow
// from the rank-2 structure of (1 -+ gamma_nu).  Every real component is one FMA.
template <int NU, bool FWD, typename R>
__device__ __forceinline__ void accumulate(cpx<R> acc[12], const cpx<R> chi[6], R coef)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cpx<R> h0 = chi[c], h1 = chi[3 + c];
        acc[c] = add_ph<kP1>(acc[c], coef, h0);
        acc[3 + c] = add_ph<kP1>(acc[3 + c], coef, h1);
        if constexpr (NU == 0) {
            acc[6 + c] = FWD ? add_ph<kPI>(acc[6 + c], coef, h1) : add_ph<kMI>(acc[6 + c], coef, h1);
            acc[9 + c] = FWD ? add_ph<kPI>(acc[9 + c], coef, h0) : add_ph<kMI>(acc[9 + c], coef, h0);
        } else if constexpr (NU == 1) {
            acc[6 + c] = FWD ? add_ph<kM1>(acc[6 + c], coef, h1) : add_ph<kP1>(acc[6 + c], coef, h1);
            acc[9 + c] = FWD ? add_ph<kP1>(acc[9 + c], coef, h0) : add_ph<kM1>(acc[9 + c], coef, h0);
        } else if constexpr (NU == 2) {
            acc[6 + c] = FWD ? add_ph<kPI>(acc[6 + c], coef, h0) : add_ph<kMI>(acc[6 + c], coef, h0);
            acc[9 + c] = FWD ? add_ph<kMI>(acc[9 + c], coef, h1) : add_ph<kPI>(acc[9 + c], coef, h1);
        } else {
            acc[6 + c] = FWD ? add_ph<kM1>(acc[6 + c], coef, h0) : add_ph<kP1>(acc[6 + c], coef, h0);
            acc[9 + c] = FWD ? add_ph<kM1>(acc[9 + c], coef, h1) : add_ph<kP1>(acc[9 + c], coef, h1);
        }
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
            cpx<R> s = cmul_f<ADJ>(ADJ ? u[a] : u[a * 3], h[3 * v]);
#pragma unroll
            for (int b = 1; b < 3; ++b) cmac_f<ADJ>(s, ADJ ? u[b * 3 + a] : u[a * 3 + b], h[3 * v + b]);
            chi[3 * v + a] = s;
        }
}

template <typename R>
using SpT = typename SpinorStore<R>::type;

// Output side of one site: gamma5 on the result, the epilogue
// out = a * in_scale * Op(in) + b * z, the store, and the site's terms of the
// partial sums conj(w) . out and ||out||^2 (FP64).  The scales are real unless
// in_scale / b_dev / Im b say otherwise (wave-uniform branches), and a dot
// partner equal to z is not read twice.
template <typename R, bool kEpi, bool kDot>
__device__ __forceinline__ void finish_site(cpx<R> (&acc)[12], const RhsParams &Q, int S, int s, double &dr,
                                            double &di, double &dn)
{
    const R s5o = static_cast<R>(Q.s5_out);
    cpx<R> zz[12];
    if constexpr (!kEpi) {
#pragma unroll
        for (int k = 6; k < 12; ++k) acc[k] = s5o * acc[k];
    } else {
        if (Q.in_scale) {
            const z64 t = *Q.in_scale;
            const cpx<R> sc = {static_cast<R>(Q.a * t.r), static_cast<R>(Q.a * t.i)};
            const cpx<R> sl = {s5o * sc.r, s5o * sc.i};
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = cmul_f<false>(k < 6 ? sc : sl, acc[k]);
        } else {
            const R a = static_cast<R>(Q.a), al = s5o * a;
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = (k < 6 ? a : al) * acc[k];
        }
        if (Q.z) {
            load_spinor(static_cast<const SpT<R> *>(Q.z), S, s, zz);
            if (!Q.b_dev && Q.b.i == 0.0) {
                const R b = static_cast<R>(Q.b.r);
#pragma unroll
                for (int k = 0; k < 12; ++k) acc[k] = add_ph<kP1>(acc[k], b, zz[k]);
            } else {
                z64 bb = Q.b;
                if (Q.b_dev) {
                    const z64 t = *Q.b_dev;
                    bb = {bb.r * t.r - bb.i * t.i, bb.r * t.i + bb.i * t.r};
                }
                const cpx<R> b = {static_cast<R>(bb.r), static_cast<R>(bb.i)};
#pragma unroll
                for (int k = 0; k < 12; ++k) cmac_f<false>(acc[k], b, zz[k]);
            }
        }
    }
    if (SGN_NT_OUT)
        store_spinor_nt(static_cast<SpT<R> *>(Q.out), S, s, acc);
    else
        store_spinor(static_cast<SpT<R> *>(Q.out), S, s, acc);
    if constexpr (kDot) {
        if (Q.w) {
            cpx<R> ww[12];
            if (kEpi && Q.w == Q.z) {
#pragma unroll
                for (int k = 0; k < 12; ++k) ww[k] = zz[k];
            } else {
                load_spinor(static_cast<const SpT<R> *>(Q.w), S, s, ww);
            }
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
            project<NU, true>(p, h, static_cast<R>(P.rhs[r].s5_in));
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
            project<NU, false>(p, h, static_cast<R>(P.rhs[r].s5_in));
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
            finish_site<R, kEpi, kDot>(acc[r], P.rhs[r], P.S, s, dr[r], di[r], dn[r]);
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

// largest block of the staged kernel (the LDS budget allows at most 64512/192 = 336 FP64 and
// 672 FP32 sites): FP64 needs ~180 VGPRs, so at most 2 waves per SIMD; the FP32 bound leaves up
// to 168 VGPRs for the multi-RHS form that holds every link of a site in registers
template <typename R> constexpr int kStagedMaxThreads = sizeof(R) == 8 ? 512 : 704;
// the multi-RHS form with the links in registers (FP16 links): 8 waves per block at most, so
// up to 256 VGPRs (two waves per SIMD)
constexpr int kRegsMaxThreads = 512;

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

// neighbour spinor n of right-hand side Q: from LDS when it belongs to this block
// (stored already multiplied by the input gamma5 sign), else from memory.  Returns
// the gamma5 sign the projection still has to apply to the lower spins.
template <typename R>
__device__ __forceinline__ R fetch_neighbour(const RhsParams &Q, const StencilParams &P, const SpT<R> *lds, int base,
                                             int n, cpx<R> p[12])
{
    const int B = P.blk_sites, NB = B * P.tslices;
    int ln = n - base;
    if ((unsigned)ln < (unsigned)B) {
        lds_load_spinor<R>(lds, NB, ln, p);
        return R(1);
    }
    if (P.tslices == 2) {  // the brick's second slice (uniform branch)
        ln = n - base - P.stride[3];
        if ((unsigned)ln < (unsigned)B) {
            lds_load_spinor<R>(lds, NB, B + ln, p);
            return R(1);
        }
    }
    load_spinor(static_cast<const SpT<R> *>(Q.in), P.S, n, p);
    return static_cast<R>(Q.s5_in);
}

// The eight links a site needs (U_nu(x) and U_nu(x - nu) for nu = 0..3, entry 2 nu + d),
// loaded once in their stored two-row form and shared by every right-hand side of the
// block (kRegs), or read from memory at each hop (kRegs false: L2 serves the repeats).
template <typename R, typename LT, bool kRegs>
struct SiteLinks {
    LT e[kRegs ? 8 : 1][kRegs ? 6 : 1];

    __device__ __forceinline__ void load(const StencilParams &P, int s, const int (&c)[4])
    {
        if constexpr (kRegs) {
            const LT *U = static_cast<const LT *>(P.links);
#pragma unroll
            for (int nu = 0; nu < 4; ++nu) {
                const int L = P.L[nu], st = P.stride[nu];
                const int nb = c[nu] == 0 ? s + (L - 1) * st : s - st;
                const LT *b = U + (size_t)nu * 6 * P.S;
                // temporal gauge: the unit time links are neither loaded nor used
                const bool fwd = !(nu == 3 && P.tgauge && c[3] != L - 1), bwd = !(nu == 3 && P.tgauge && c[3] != 0);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    if (fwd) e[2 * nu][k] = ld_off(b + (size_t)k * P.S, (uint32_t)s * (uint32_t)sizeof(LT));
                    if (bwd) e[2 * nu + 1][k] = ld_off(b + (size_t)k * P.S, (uint32_t)nb * (uint32_t)sizeof(LT));
                }
            }
        }
    }

    // link K = 2 nu + d as a full 3x3 matrix; n: the site it belongs to (s, or x - nu)
    template <int K>
    __device__ __forceinline__ void get(const StencilParams &P, int n, cpx<R> u[9]) const
    {
        if constexpr (kRegs) {
#pragma unroll
            for (int k = 0; k < 6; ++k) u[k] = to_cpx<R>(e[K][k]);
            su3_third_row(u);
        } else {
            load_link<R>(static_cast<const LT *>(P.links), P.S, P.link_ne, K / 2, n, u);
        }
    }
};

template <int NU, typename R, typename LT, bool kRegs>
__device__ __forceinline__ void hop_pair_staged(cpx<R> (&acc)[12], const StencilParams &P, const RhsParams &Q,
                                                const SpT<R> *lds, int base, int s, int coord,
                                                const SiteLinks<R, LT, kRegs> &lk)
{
    const int L = P.L[NU], st = P.stride[NU];
    const R kap = static_cast<R>(P.kappa);
    cpx<R> u[9];
    {
        const bool wrap = coord == L - 1;
        const int n = wrap ? s - (L - 1) * st : s + st;
        const R bcf = wrap ? static_cast<R>(P.bcf[NU]) : R(1);
        cpx<R> p[12], h[6], chi[6];
        const bool unit = NU == 3 && P.tgauge && !wrap;  // temporal gauge: U_t(x) = 1
        if (!unit) lk.template get<2 * NU>(P, s, u);
        const R s5 = fetch_neighbour<R>(Q, P, lds, base, n, p);
        project<NU, true>(p, h, s5);
        if (unit) {
#pragma unroll
            for (int k = 0; k < 6; ++k) chi[k] = h[k];
        } else {
            link_mul<false>(u, h, chi);
        }
        const R w = NU == 3 ? static_cast<R>(Q.wf_t) : R(1);
        accumulate<NU, true>(acc, chi, -kap * w * bcf);
    }
    pin(acc);
    {
        const bool wrap = coord == 0;
        const int n = wrap ? s + (L - 1) * st : s - st;
        const R bcb = wrap ? static_cast<R>(P.bcf[NU]) : R(1);
        cpx<R> p[12], h[6], chi[6];
        const bool unit = NU == 3 && P.tgauge && !wrap;  // temporal gauge: U_t(x - t) = 1
        if (!unit) lk.template get<2 * NU + 1>(P, n, u);
        const R s5 = fetch_neighbour<R>(Q, P, lds, base, n, p);
        project<NU, false>(p, h, s5);
        if (unit) {
#pragma unroll
            for (int k = 0; k < 6; ++k) chi[k] = h[k];
        } else {
            link_mul<true>(u, h, chi);
        }
        const R w = NU == 3 ? static_cast<R>(Q.wb_t) : R(1);
        accumulate<NU, false>(acc, chi, -kap * w * bcb);
    }
    pin(acc);
}

// One block: B sites for each right-hand side in turn (kMulti: the P.nrhs right-hand sides
// of P's group, all on P's lattice; else the single one, P.rhs[0]); the block's own spinors of
// the current right-hand side are staged in LDS.  The single form indexes P.rhs only with
// constants: P is then a kernel argument, and a runtime index into it would copy it to private
// memory.
template <typename R, typename LT, bool kEpi, bool kDot, bool kRegs, bool kMulti>
__device__ __forceinline__ void staged_body(const StencilParams &P, const int bx)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SpT<R> *lds = reinterpret_cast<SpT<R> *>(smem_raw);
    if (bx >= P.nblk_sites) {  // padding of the component arrays: keep it zero
        const int s = P.V + (bx - P.nblk_sites) * (int)blockDim.x + (int)threadIdx.x;
        const int nr = kMulti ? P.nrhs : 1;
        for (int r = 0; r < nr; ++r) {
            const RhsParams &Q = P.rhs[kMulti ? r : 0];
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
        }
        return;
    }
    const int B = P.blk_sites, NB = B * P.tslices;
    int blk;
    if (P.sched_T > 0) {
        // XCD k owns the t-slab [k T, (k+1) T) of sched_R blocks per t-slice (per pair of
        // t-slices for bricks) and walks it in strips of W consecutive blocks with t fastest, so
        // the t-neighbours of a block run on the same XCD at about the same time
        const int W = SGN_STAGED_STRIP;
        const int k = bx % 8, j = bx / 8;
        const int per_strip = P.sched_T * W;
        const int strip = j / per_strip, rem = j - strip * per_strip;
        const int tl = rem / W, wi = rem - tl * W;
        blk = (k * P.sched_T + tl) * P.sched_R + strip * W + wi;
    } else {
        blk = SGN_XCD_REMAP ? xcd_block(bx, P.nblk_sites) : bx;
    }
    // first site of the block: B consecutive sites of one t-slice, for bricks the same B sites
    // of the next slice too (threads B.. 2B-1); blocks tile the V sites exactly
    int base;
    if (P.tslices == 2) {
        const int nreg = P.stride[3] / B, g = blk / nreg;
        base = 2 * g * P.stride[3] + (blk - g * nreg) * B;
    } else {
        base = blk * B;
    }
    const int i = threadIdx.x;
    const bool valid = i < NB;
    const int s = i < B ? base + i : base + P.stride[3] + (i - B);
    int c[4] = {0, 0, 0, 0};
    if (valid) {
        c[0] = s % P.L[0];
        int q = s / P.L[0];
        c[1] = q % P.L[1];
        q /= P.L[1];
        c[2] = q % P.L[2];
        c[3] = q / P.L[2];
    }
    SiteLinks<R, LT, kRegs> lk;
    if (valid) lk.load(P, s, c);
    const int nr = kMulti ? P.nrhs : 1;
    for (int r = 0; r < nr; ++r) {
        const RhsParams &Q = P.rhs[kMulti ? r : 0];
        if (r > 0) __syncthreads();  // the previous right-hand side's LDS reads are done
        cpx<R> acc[12];
        if (valid) {
            load_spinor(static_cast<const SpT<R> *>(Q.in), P.S, s, acc);
            const R s5 = static_cast<R>(Q.s5_in);
#pragma unroll
            for (int k = 6; k < 12; ++k) acc[k] = s5 * acc[k];
            lds_store_spinor<R>(lds, NB, i, acc);
        }
        __syncthreads();
        double dr = 0.0, di = 0.0, dn = 0.0;
        if (valid) {
            hop_pair_staged<0, R, LT, kRegs>(acc, P, Q, lds, base, s, c[0], lk);
            hop_pair_staged<1, R, LT, kRegs>(acc, P, Q, lds, base, s, c[1], lk);
            hop_pair_staged<2, R, LT, kRegs>(acc, P, Q, lds, base, s, c[2], lk);
            hop_pair_staged<3, R, LT, kRegs>(acc, P, Q, lds, base, s, c[3], lk);
            finish_site<R, kEpi, kDot>(acc, Q, P.S, s, dr, di, dn);
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
}

// Waves per SIMD the compiler must allow the single-RHS staged kernel: with FP16 links 5 (at most 96
// VGPRs; the epilogue form spills a few bytes and still gains 3% inside the solves); otherwise what
// the largest block already implies (FP32 and FP64 lost time to spills when pushed further).
template <typename R, typename LT>
constexpr int kStagedWaves = std::is_same<LT, __half2>::value ? 5 : (sizeof(R) == 8 ? 2 : 3);

template <typename R, typename LT, bool kEpi, bool kDot>
__global__ void __launch_bounds__(kStagedMaxThreads<R>) __attribute__((amdgpu_waves_per_eu(kStagedWaves<R, LT>)))
    stencil_staged_kernel(StencilParams P)
{
    staged_body<R, LT, kEpi, kDot, false, false>(P, (int)blockIdx.x);
}

// Batched form: blockIdx.y selects one of several independent applications
// (own lattice, right-hand sides and epilogues) whose parameters live in device
// memory.  gridDim.x is a multiple of 8, so the XCD of block (x, y) is x mod 8 as
// in the single form.
template <typename R, typename LT, bool kEpi, bool kDot, bool kRegs>
__global__ void __launch_bounds__(kRegs ? kRegsMaxThreads : kStagedMaxThreads<R>)
    stencil_staged_batch(const StencilParams *__restrict__ plist)
{
    const StencilParams &P = plist[blockIdx.y];
    if ((int)blockIdx.x >= P.nblk_total) return;
    staged_body<R, LT, kEpi, kDot, kRegs, true>(P, (int)blockIdx.x);
}

template <typename R, typename LT>
void launch_staged(const StencilParams &P, int nblk, int threads, size_t lds, bool epi, bool dot, hipStream_t s,
                   const LaunchStamp &ev)
{
    dim3 g(nblk), b(threads);
    if (dot)
        launch_k(ev, stencil_staged_kernel<R, LT, true, true>, g, b, (uint32_t)lds, s, P);
    else if (epi)
        launch_k(ev, stencil_staged_kernel<R, LT, true, false>, g, b, (uint32_t)lds, s, P);
    else
        launch_k(ev, stencil_staged_kernel<R, LT, false, false>, g, b, (uint32_t)lds, s, P);
}

template <typename R, typename LT, int NR>
void launch_typed(const StencilParams &P, int nblk, bool epi, bool dot, hipStream_t s, const LaunchStamp &ev)
{
    dim3 g(nblk), b(SGN_STENCIL_THREADS);
    if (dot)
        launch_k(ev, stencil_kernel<R, LT, NR, true, true>, g, b, 0u, s, P);
    else if (epi)
        launch_k(ev, stencil_kernel<R, LT, NR, true, false>, g, b, 0u, s, P);
    else
        launch_k(ev, stencil_kernel<R, LT, NR, false, false>, g, b, 0u, s, P);
}

// unstaged kernel (lattices too small for a staged block shape): one launch per right-hand side;
// a stamp is only taken for one right-hand side (one launch)
template <typename R, typename LT>
void launch_nr(const StencilParams &P, int nr, int nblk, bool epi, bool dot, hipStream_t s, const LaunchStamp &ev)
{
    if (nr == 1) {
        launch_typed<R, LT, 1>(P, nblk, epi, dot, s, ev);
        return;
    }
    for (int r = 0; r < nr; ++r) {
        StencilParams Q = P;
        Q.rhs[0] = P.rhs[r];
        Q.nrhs = 1;
        launch_typed<R, LT, 1>(Q, nblk, epi, dot, s, LaunchStamp{});
    }
}

}  // namespace

namespace {

// Block shape of the staged kernel: B sites of whole x-rows (whole x-y planes
// when they fit the LDS budget), B dividing V; not used when B < 64.
struct StagedPlan {
    bool ok = false;
    int B = 0, T = 1, threads = 0, nblk_sites = 0, nblk = 0;  // B sites per t-slice, T slices per block
    size_t lds = 0;
};

// max_threads > 0 caps the block (the register-link multi-RHS form), max_sites > 0 the sites of
// a block (a tuned shape); tslices = 2 asks for bricks of two t-slices (even L_t; B then divides
// one slice, so a brick never straddles a time boundary)
StagedPlan staged_plan(const Lattice &lat, sgn_prec p, int max_threads = 0, int max_sites = 0, int tslices = 1)
{
    StagedPlan pl;
    if (!SGN_STENCIL_LDS) return pl;
    const int T = tslices == 2 ? 2 : 1;
    if (T == 2 && lat.L[3] % 2) return pl;
    const int64_t site_bytes = p == SGN_PREC_F64 ? 192 : 96;
    int64_t tmax = p == SGN_PREC_F64 ? kStagedMaxThreads<double> : kStagedMaxThreads<float>;
    if (max_threads > 0) tmax = std::min<int64_t>(tmax, max_threads);
    if (max_sites > 0) tmax = std::min<int64_t>(tmax, max_sites);
    const int64_t bmax = std::min<int64_t>(tmax, SGN_LDS_MAXBYTES / site_bytes) / T;
    const int64_t Lx = lat.L[0], A = (int64_t)lat.L[0] * lat.L[1];
    const int64_t nplane = (int64_t)lat.L[2] * (T == 2 ? 1 : lat.L[3]);
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
    if (B * T < 64) return pl;
    pl.ok = true;
    pl.B = (int)B;
    pl.T = T;
    pl.threads = (int)((B * T + 63) / 64 * 64);
    pl.nblk_sites = (int)(lat.V / (B * T));
    const int64_t pad = lat.S > lat.V ? (lat.S - lat.V + pl.threads - 1) / pl.threads : 0;
    pl.nblk = pl.nblk_sites + (int)pad;
    pl.lds = (size_t)B * T * site_bytes;
    return pl;
}

}  // namespace

// An upper bound of the blocks of any stencil launch on lat, whatever shape is chosen (tuned or
// default): every staged block holds at least 64 sites, the unstaged kernel 256, and the padding
// sites [V, S) take blocks of at least 64 threads.  Sizes the per-block partial sums.
int dslash_blocks(const Lattice &lat)
{
    const int64_t valid = (lat.V + 63) / 64;
    const int64_t pad = lat.S > lat.V ? (lat.S - lat.V + 63) / 64 : 0;
    return (int)(valid + pad);
}

namespace {

// Everything about one stencil application except the launch itself.
struct PreparedStencil {
    StencilParams P{};
    StagedPlan pl;
    int nblk = 0;       // blocks of the launch (= partials written when dotting)
    double bytes = 0.0;         // algorithmic bytes (links as nine entries) and flops
    double flops = 0.0;
    double bytes_stored = 0.0;  // bytes in the stored format (two-row links where the lattice keeps them)
    bool epi = false, dot = false;
};

// max_threads > 0 caps the staged block (the register-link multi-RHS form)
PreparedStencil prepare_stencil(const Lattice &lat, sgn_prec p, int nr, const OpSpec *op, const void *const *in,
                                void *const *out, const Epilogue *ep, int max_threads = 0)
{
    if (nr < 1 || nr > kMaxRhs) throw Failure{SGN_ERR_INVALID, "stencil: 1..16 right-hand sides per launch"};
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
        // an epilogue operand counts once: a dot partner equal to z is not read again
        extra_bytes += (ep[r].z ? sb : 0.0) + (ep[r].w && ep[r].w != ep[r].z ? sb : 0.0);
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
    // site once (shared by the right-hand sides) as nine complex entries, plus the
    // epilogue operands; 1368 flop per site and right-hand side for the stencil itself
    P.link_ne = lat.link_ne;
    P.tgauge = 0;
    const double eb = (p == SGN_PREC_F64) ? 16.0 : (p == SGN_PREC_F32 ? 8.0 : 4.0);
    ps.bytes = (2 * sb * nr + 4 * 9 * eb + extra_bytes) * lat.V;
    ps.bytes_stored = (2 * sb * nr + 4 * lat.link_ne * eb + extra_bytes) * lat.V;
    ps.flops = (1368.0 * nr + extra_flops) * lat.V;
    P.nrhs = nr;
    P.tslices = 1;
    {
        const Context::TunedShape ts = lat.ctx->tuned_shape(lat.L, p, nr > 1);
        if (!ts.unstaged) {
            ps.pl = staged_plan(lat, p, max_threads, ts.max_sites, ts.tslices);
            if (!ps.pl.ok && ts.tslices == 2) ps.pl = staged_plan(lat, p, max_threads, ts.max_sites, 1);
        }
    }
    if (ps.pl.ok) {
        P.blk_sites = ps.pl.B;
        P.tslices = ps.pl.T;
        P.nblk_sites = ps.pl.nblk_sites;
        ps.nblk = ps.pl.nblk;
        P.sched_T = P.sched_R = 0;
        const int64_t v3 = (int64_t)lat.L[0] * lat.L[1] * lat.L[2];
        const int tg = lat.L[3] / ps.pl.T;  // t-slices, or pairs of them for bricks
        if (SGN_STAGED_STRIP > 0 && v3 % ps.pl.B == 0 && tg % 8 == 0 && (v3 / ps.pl.B) % SGN_STAGED_STRIP == 0) {
            P.sched_T = tg / 8;
            P.sched_R = (int)(v3 / ps.pl.B);
        }
    }
    P.nblk_total = ps.nblk;
    if (lat.gauge && ps.pl.ok) {  // the staged kernel reads the time links of the last slice only
        P.tgauge = 1;
        ps.bytes_stored -= (1.0 - 1.0 / lat.L[3]) * lat.link_ne * ((p == SGN_PREC_F64) ? 16.0 : (p == SGN_PREC_F32 ? 8.0 : 4.0)) * lat.V;
    }
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

template <typename R, typename LT, bool kRegs>
void launch_staged_batch_r(const StencilParams *dev, int count, int gx, int threads, size_t lds, bool epi, bool dot,
                           hipStream_t s, const LaunchStamp &ev)
{
    dim3 g(gx, count), b(threads);
    if (dot)
        launch_k(ev, stencil_staged_batch<R, LT, true, true, kRegs>, g, b, (uint32_t)lds, s, dev);
    else if (epi)
        launch_k(ev, stencil_staged_batch<R, LT, true, false, kRegs>, g, b, (uint32_t)lds, s, dev);
    else
        launch_k(ev, stencil_staged_batch<R, LT, false, false, kRegs>, g, b, (uint32_t)lds, s, dev);
}

template <typename R, typename LT>
void launch_staged_batch(const StencilParams *dev, int count, int gx, int threads, size_t lds, bool epi, bool dot,
                         bool regs, hipStream_t s, const LaunchStamp &ev)
{
    if constexpr (std::is_same<LT, __half2>::value) {
        if (regs) {
            launch_staged_batch_r<R, LT, true>(dev, count, gx, threads, lds, epi, dot, s, ev);
            return;
        }
    }
    launch_staged_batch_r<R, LT, false>(dev, count, gx, threads, lds, epi, dot, s, ev);
}

}  // namespace

int dslash_launch_multi(const Lattice &lat, sgn_prec p, int nr, const OpSpec *op, const void *const *in,
                        void *const *out, const Epilogue *ep, hipStream_t s)
{
    const PreparedStencil ps = prepare_stencil(lat, p, nr, op, in, out, ep);
    if (nr > 1 && ps.pl.ok) {
        // several right-hand sides: the batched form, one group, parameters in device memory
        // (the lattice's batch object: they are uploaded when they change, after the device has
        // finished the launches that read the previous ones)
        std::vector<StencilJob> jobs(nr);
        for (int r = 0; r < nr; ++r) jobs[r] = StencilJob{&lat, op[r], in[r], out[r], ep[r]};
        if (!lat.multi) lat.multi = std::make_shared<StencilBatch>();
        lat.multi->prepare(jobs, p);
        lat.multi->launch(s);
        return ps.nblk;
    }
    // one launch unless the unstaged kernel runs several right-hand sides
    const int prof = lat.ctx->prof_start(s, kclass(p), ps.pl.ok || nr == 1);
    const LaunchStamp ev = lat.ctx->prof_stamp(prof);
    switch (p) {
    case SGN_PREC_F64:
        if (ps.pl.ok)
            launch_staged<double, double2>(ps.P, ps.nblk, ps.pl.threads, ps.pl.lds, ps.epi, ps.dot, s, ev);
        else
            launch_nr<double, double2>(ps.P, nr, ps.nblk, ps.epi, ps.dot, s, ev);
        break;
    case SGN_PREC_F32:
        if (ps.pl.ok)
            launch_staged<float, float2>(ps.P, ps.nblk, ps.pl.threads, ps.pl.lds, ps.epi, ps.dot, s, ev);
        else
            launch_nr<float, float2>(ps.P, nr, ps.nblk, ps.epi, ps.dot, s, ev);
        break;
    default:
        if (ps.pl.ok)
            launch_staged<float, __half2>(ps.P, ps.nblk, ps.pl.threads, ps.pl.lds, ps.epi, ps.dot, s, ev);
        else
            launch_nr<float, __half2>(ps.P, nr, ps.nblk, ps.epi, ps.dot, s, ev);
        break;
    }
    SGN_HIP(hipGetLastError());
    lat.ctx->prof_stop(prof, s, kclass(p), ps.bytes, ps.flops, false, ps.bytes_stored);
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
    bytes_ = flops_ = bytes_stored_ = 0.0;
    // applications on the same lattice become multi-RHS groups (right-hand sides sharing every
    // link load); the groups are the launch's blockIdx.y.  A group's block walks its right-hand
    // sides one after another, so the group size is the largest (up to kMaxRhs) that still leaves
    // the launch 1024 blocks of sites (four per CU), or as many as groups of one would: small
    // lattices trade link sharing for parallelism
    int gsize = kMaxRhs;
    {
        std::vector<const Lattice *> lats;
        std::vector<int64_t> cnt, per;
        for (const StencilJob &j : jobs) {
            size_t l = 0;
            while (l < lats.size() && lats[l] != j.lat) ++l;
            if (l == lats.size()) {
                lats.push_back(j.lat);
                cnt.push_back(0);
                const Context::TunedShape ts = j.lat->ctx->tuned_shape(j.lat->L, p, true);
                const StagedPlan pl = staged_plan(*j.lat, p, 0, ts.max_sites, ts.tslices);
                per.push_back(pl.ok ? pl.nblk_sites : (j.lat->V + 255) / 256);
            }
            ++cnt[l];
        }
        auto blocks = [&](int g) {
            int64_t b = 0;
            for (size_t l = 0; l < lats.size(); ++l) b += (cnt[l] + g - 1) / g * per[l];
            return b;
        };
        const int64_t want = std::min<int64_t>(1024, blocks(1));
        while (gsize > 1 && blocks(gsize) < want) --gsize;
    }
    std::vector<std::vector<size_t>> groups;
    for (size_t k = 0; k < jobs.size(); ++k) {
        size_t g = 0;
        for (; g < groups.size(); ++g)
            if (jobs[groups[g][0]].lat == jobs[k].lat && (int)groups[g].size() < gsize) break;
        if (g == groups.size()) groups.emplace_back();
        groups[g].push_back(k);
    }
    // links in registers (FP16 two-row links, some group with several right-hand sides, and the
    // environment does not ask for re-reads: SGN_MULTI_LINK_REGS=0)
    regs_ = p == SGN_PREC_F32_H16;
    bool multi = false;
    for (size_t g = 0; g < groups.size(); ++g) {
        multi = multi || groups[g].size() > 1;
        regs_ = regs_ && jobs[groups[g][0]].lat->link_ne == 6;
    }
    {
        const char *e = std::getenv("SGN_MULTI_LINK_REGS");
        const int tuned = groups.empty() ? -1 : jobs[groups[0][0]].lat->ctx->tuned_shape(jobs[groups[0][0]].lat->L, p, true).regs;
        regs_ = regs_ && multi && !(e && e[0] == '0') && tuned != 0;
    }
    std::vector<StencilParams> host(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        const int nr = (int)groups[g].size();
        std::vector<OpSpec> op(nr);
        std::vector<const void *> in(nr);
        std::vector<void *> out(nr);
        std::vector<Epilogue> ep(nr);
        for (int r = 0; r < nr; ++r) {
            const StencilJob &j = jobs[groups[g][r]];
            op[r] = j.op;
            in[r] = j.in;
            out[r] = j.out;
            ep[r] = j.ep;
        }
        const Lattice &lat = *jobs[groups[g][0]].lat;
        const PreparedStencil ps = prepare_stencil(lat, p, nr, op.data(), in.data(), out.data(), ep.data(),
                                                   regs_ ? kRegsMaxThreads : 0);
        host[g] = ps.P;
        for (size_t k : groups[g]) nblk_[k] = ps.nblk;
        batched_ = batched_ && ps.pl.ok;
        epi_ = epi_ || ps.epi;
        dot_ = dot_ || ps.dot;
        gx_ = std::max(gx_, ps.nblk);
        threads_ = std::max(threads_, ps.pl.threads);
        lds_ = std::max(lds_, ps.pl.lds);
        bytes_ += ps.bytes;
        bytes_stored_ += ps.bytes_stored;
        flops_ += ps.flops;
    }
    ngroups_ = (int)groups.size();
    gx_ = (gx_ + 7) / 8 * 8;
    if (!batched_) return;
    const size_t need = sizeof(StencilParams) * host.size();
    // unchanged parameters stay on the device; new ones wait until no launch reads the old
    if (need == uploaded_.size() && std::memcmp(uploaded_.data(), host.data(), need) == 0) return;
    SGN_HIP(hipDeviceSynchronize());
    if (need > dev_bytes_) {
        if (dev_) SGN_HIP(hipFree(dev_));
        dev_ = nullptr;
        dev_bytes_ = 0;
        if (hipMalloc(&dev_, need) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "stencil batch parameters"};
        dev_bytes_ = need;
    }
    SGN_HIP(hipMemcpy(dev_, host.data(), need, hipMemcpyHostToDevice));
    uploaded_.assign(reinterpret_cast<const char *>(host.data()), reinterpret_cast<const char *>(host.data()) + need);
}

void StencilBatch::launch(hipStream_t s) const
{
    if (jobs_.empty()) return;
    if (!batched_) {  // some lattice has no staged block shape: one launch per application
        for (const StencilJob &j : jobs_) dslash_launch(*j.lat, prec_, j.op, j.in, j.out, j.ep, s);
        return;
    }
    Context *ctx = jobs_[0].lat->ctx;
    const int prof = ctx->prof_start(s, kclass(prec_), true);
    const LaunchStamp ev = ctx->prof_stamp(prof);
    const StencilParams *d = static_cast<const StencilParams *>(dev_);
    const int cnt = ngroups_;
    switch (prec_) {
    case SGN_PREC_F64:
        launch_staged_batch<double, double2>(d, cnt, gx_, threads_, lds_, epi_, dot_, false, s, ev);
        break;
    case SGN_PREC_F32:
        launch_staged_batch<float, float2>(d, cnt, gx_, threads_, lds_, epi_, dot_, regs_, s, ev);
        break;
    default: launch_staged_batch<float, __half2>(d, cnt, gx_, threads_, lds_, epi_, dot_, regs_, s, ev); break;
    }
    SGN_HIP(hipGetLastError());
    ctx->prof_stop(prof, s, kclass(prec_), bytes_, flops_, false, bytes_stored_);
}

int dslash_launch(const Lattice &lat, sgn_prec p, const OpSpec &op, const void *in, void *out,
                  const Epilogue &ep, hipStream_t s)
{
    return dslash_launch_multi(lat, p, 1, &op, &in, &out, &ep, s);
}

}  // namespace sgn

// ----------------------------------------------------------------------------- no-allocation scratch
// Staging of the two fields of wilson_apply_noalloc: one file-scope device array, a copy of
// which every GPU holds from the time the library's code is loaded on it until the process
// ends.  Host code never passes the array's name (a host-side stand-in) to a kernel or copy:
// noalloc_scratch() takes its address on each device once, with that device current, and
// kernels receive that address.
static __device__ __align__(256) unsigned char scratch[SGN_NOALLOC_MAX_BYTES];

namespace sgn {

void *noalloc_scratch(int device)
{
    static std::mutex mu;
    static std::map<int, void *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) return it->second;
    int cur = -1;
    SGN_HIP(hipGetDevice(&cur));
    SGN_REQUIRE(cur == device, "no-allocation scratch: the device must be current");
    void *ptr = nullptr;
    SGN_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    SGN_REQUIRE(ptr != nullptr, "no-allocation scratch: no device address");
    addr[device] = ptr;
    return ptr;
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

extern "C" sgn_status wilson_apply_noalloc(sgn_lattice l, double mu, const void *in, void *out, sgn_prec p,
                                           unsigned flags, void *stream)
{
    return guard([&] {
        SGN_REQUIRE(l != nullptr && in != nullptr && out != nullptr, "wilson_apply_noalloc: null argument");
        SGN_REQUIRE(in != out, "wilson_apply_noalloc: in and out must differ");
        SGN_REQUIRE(std::isfinite(mu), "wilson_apply_noalloc: mu is not finite");
        SGN_REQUIRE(p == SGN_PREC_F64 || p == SGN_PREC_F32 || p == SGN_PREC_F32_H16,
                    "wilson_apply_noalloc: unknown precision");
        Lattice &lat = *as_lattice(l);
        SGN_HIP(hipSetDevice(lat.ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        OpSpec op;
        op.mu = mu;
        op.g5_out = !(flags & SGN_NO_GAMMA5);
        Epilogue ep;
        if (flags & SGN_INTERNAL_LAYOUT) {  // no staging needed
            dslash_launch(lat, p, op, in, out, ep, s);
            return;
        }
        const size_t bytes = spinor_bytes(lat.S, p);
        const size_t off = (bytes + 255) / 256 * 256;  // second field 256-byte aligned
        if (off + bytes > (size_t)SGN_NOALLOC_MAX_BYTES)
            throw Failure{SGN_ERR_INVALID, "wilson_apply_noalloc: the lattice needs " + std::to_string(off + bytes) +
                                               " staging bytes, more than SGN_NOALLOC_MAX_BYTES = " +
                                               std::to_string((size_t)SGN_NOALLOC_MAX_BYTES)};
        SGN_REQUIRE(lat.ctx->noalloc != nullptr, "wilson_apply_noalloc: scratch address not set up");
        char *stage_in = static_cast<char *>(lat.ctx->noalloc);
        char *stage_out = stage_in + off;
        pack_spinor(lat, in, stage_in, p, s);
        dslash_launch(lat, p, op, stage_in, stage_out, ep, s);
        unpack_spinor(lat, stage_out, out, p, s);
    });
}

extern "C" sgn_status sgn_autotune(sgn_lattice l, sgn_prec p, int nrhs, int reps, sgn_tune_candidate *out,
                                   int max_out, int *n_out, void *stream)
{
    return guard([&] {
        SGN_REQUIRE(l != nullptr, "sgn_autotune: null lattice");
        SGN_REQUIRE(p == SGN_PREC_F64 || p == SGN_PREC_F32 || p == SGN_PREC_F32_H16, "sgn_autotune: unknown precision");
        SGN_REQUIRE(nrhs >= 1 && nrhs <= kMaxRhs, "sgn_autotune: nrhs must be 1..16");
        SGN_REQUIRE(max_out >= 0 && (max_out == 0 || out != nullptr), "sgn_autotune: bad output array");
        Lattice &lat = *as_lattice(l);
        Context &ctx = *lat.ctx;
        SGN_HIP(hipSetDevice(ctx.device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (reps <= 0) reps = 20;
        const bool multi = nrhs > 1;
        const std::vector<int> key = {lat.L[0], lat.L[1], lat.L[2], lat.L[3], (int)p, multi ? 1 : 0};
        // candidate shapes: distinct blocks of the staged plan under decreasing site caps, as one
        // t-slice or as bricks of two, and for several right-hand sides with FP16 two-row links both
        // link modes
        struct Cand {
            int cap, B, T, regs;
            double us;
            int unstaged;
        };
        std::vector<Cand> cands;
        if (!multi) cands.push_back({0, 0, 1, -1, 0.0, 1});  // the unstaged kernel
        const bool can_regs = multi && p == SGN_PREC_F32_H16 && lat.link_ne == 6;
        for (int regs : can_regs ? std::vector<int>{1, 0} : std::vector<int>{-1}) {
            for (int T : {1, 2}) {
                std::vector<int> seen;
                for (int cap : {0, 576, 432, 384, 288, 192, 96}) {
                    const StagedPlan pl = staged_plan(lat, p, regs == 1 ? kRegsMaxThreads : 0, cap, T);
                    if (!pl.ok && T == 2) continue;
                    const int B = pl.ok ? pl.B : 0;
                    if (std::find(seen.begin(), seen.end(), B) != seen.end()) continue;
                    seen.push_back(B);
                    cands.push_back({cap, B, pl.ok ? pl.T : 1, regs, 0.0, 0});
                }
            }
        }
        // fields: nrhs inputs (zero) and outputs in the internal layout
        const size_t bytes = spinor_bytes(lat.S, p);
        std::vector<void *> buf(2 * nrhs, nullptr);
        struct Free {
            std::vector<void *> &b;
            ~Free()
            {
                for (void *q : b)
                    if (q) (void)hipFree(q);
            }
        } freer{buf};
        for (void *&q : buf) {
            if (hipMalloc(&q, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "sgn_autotune: fields"};
            SGN_HIP(hipMemsetAsync(q, 0, bytes, s));
        }
        std::vector<OpSpec> op(nrhs);
        std::vector<Epilogue> ep(nrhs);
        std::vector<const void *> in(nrhs);
        std::vector<void *> outp(nrhs);
        for (int r = 0; r < nrhs; ++r) {
            op[r].mu = 0.2;
            in[r] = buf[r];
            outp[r] = buf[nrhs + r];
        }
        hipEvent_t e0, e1;
        SGN_HIP(hipEventCreate(&e0));
        SGN_HIP(hipEventCreate(&e1));
        const Context::TunedShape before = ctx.tuned_shape(lat.L, p, multi);
        try {
            for (Cand &c : cands) {
                ctx.tuned[key] = {c.cap, c.regs, c.T, c.unstaged};
                for (int w = 0; w < 3; ++w) dslash_launch_multi(lat, p, nrhs, op.data(), in.data(), outp.data(), ep.data(), s);
                SGN_HIP(hipEventRecord(e0, s));
                for (int k = 0; k < reps; ++k)
                    dslash_launch_multi(lat, p, nrhs, op.data(), in.data(), outp.data(), ep.data(), s);
                SGN_HIP(hipEventRecord(e1, s));
                SGN_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                SGN_HIP(hipEventElapsedTime(&ms, e0, e1));
                c.us = 1e3 * ms / reps;
            }
        } catch (...) {
            ctx.tuned[key] = before;
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        const Cand *best = &cands[0];
        for (const Cand &c : cands)
            if (c.us < best->us) best = &c;
        ctx.tuned[key] = {best->cap, best->regs, best->T, best->unstaged};
        SGN_HIP(hipDeviceSynchronize());
        const int n = std::min<int>((int)cands.size(), max_out);
        for (int k = 0; k < n; ++k)
            out[k] = {cands[k].B * cands[k].T, cands[k].regs < 0 ? 0 : cands[k].regs, cands[k].us,
                      &cands[k] == best ? 1 : 0, cands[k].T};
        if (n_out) *n_out = (int)cands.size();
    });
}

extern "C" sgn_status sgn_tune_set(sgn_lattice l, sgn_prec p, int multi, int max_sites, int t_slices,
                                   int links_in_registers)
{
    return guard([&] {
        SGN_REQUIRE(l != nullptr, "sgn_tune_set: null lattice");
        SGN_REQUIRE(p == SGN_PREC_F64 || p == SGN_PREC_F32 || p == SGN_PREC_F32_H16, "sgn_tune_set: unknown precision");
        SGN_REQUIRE(max_sites >= -1, "sgn_tune_set: max_sites must be >= -1");
        SGN_REQUIRE(t_slices == 1 || t_slices == 2, "sgn_tune_set: t_slices must be 1 or 2");
        SGN_REQUIRE(links_in_registers >= -1 && links_in_registers <= 1, "sgn_tune_set: links_in_registers is -1, 0 or 1");
        Lattice &lat = *as_lattice(l);
        const bool unstaged = max_sites == -1;
        if (!unstaged) {
            const StagedPlan pl = staged_plan(lat, p, 0, max_sites, t_slices);
            SGN_REQUIRE(pl.ok && pl.T == t_slices, "sgn_tune_set: no staged block of this shape fits the lattice");
        }
        // the parameters of earlier multi-RHS launches may still be read by the device
        SGN_HIP(hipSetDevice(lat.ctx->device));
        SGN_HIP(hipDeviceSynchronize());
        lat.ctx->tuned[{lat.L[0], lat.L[1], lat.L[2], lat.L[3], (int)p, multi ? 1 : 0}] =
            Context::TunedShape{unstaged ? 0 : max_sites, links_in_registers, t_slices, unstaged ? 1 : 0};
    });
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
