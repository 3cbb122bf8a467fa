// Device-side access to fields in the library's internal (site-fastest) layout.
//
//   spinor FP64 : [12][S] double2       component k = 3*spin + colour
//   spinor FP32 : [6][S]  float4        chunk c holds components 2c and 2c+1
//   links       : [4][9][S] of double2 / float2 / __half2, element 3*a + b of U_nu(x)
// S >= V is the lattice's padded component stride; entries s >= V are zero.
//
// Consecutive lanes read consecutive sites of the same component, so every
// wavefront-wide load is one contiguous 512 B .. 1 KiB segment.
#pragma once

#include "sgn_internal.h"

namespace sgn {

template <typename R> struct SpinorStore;
template <> struct SpinorStore<double> { using type = double2; static constexpr int chunks = 12; };
template <> struct SpinorStore<float> { using type = float4; static constexpr int chunks = 6; };

// Load/store with a wavefront-uniform base (kept in SGPRs) plus a 32-bit
// per-lane byte offset: lets the compiler use the SGPR-base addressing mode
// instead of one 64-bit VGPR address per component (which costs ~2 VGPRs per
// load in flight and made the stencil spill).
// The fields always live in device (global) memory; saying so explicitly keeps the
// accesses global_load/global_store when the pointer itself was read from memory (the
// batched launches keep their parameters in device memory).  Generic pointers would
// give flat instructions, which count against the LDS wait counter as well and so
// serialise the stencil's LDS reads behind its outstanding memory loads.
// (the host compilation pass of these device functions has no address spaces)
#if defined(__HIP_DEVICE_COMPILE__)
#define SGN_GLOBAL __attribute__((address_space(1)))
#else
#define SGN_GLOBAL
#endif

template <typename T>
__device__ __forceinline__ T ld_off(const T *__restrict__ base, uint32_t byte_off)
{
    const SGN_GLOBAL char *b = (const SGN_GLOBAL char *)base;
    return *reinterpret_cast<const SGN_GLOBAL T *>(b + byte_off);
}

template <typename T>
__device__ __forceinline__ void st_off(T *__restrict__ base, uint32_t byte_off, T v)
{
    SGN_GLOBAL char *b = (SGN_GLOBAL char *)base;
    *reinterpret_cast<SGN_GLOBAL T *>(b + byte_off) = v;
}

__device__ __forceinline__ void load_spinor(const double2 *__restrict__ p, int S, int s, cpx<double> v[12])
{
    const uint32_t off = (uint32_t)s * 16u;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 t = ld_off(p + (size_t)c * S, off);
        v[c] = {t.x, t.y};
    }
}

__device__ __forceinline__ void load_spinor(const float4 *__restrict__ p, int S, int s, cpx<float> v[12])
{
    const uint32_t off = (uint32_t)s * 16u;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        float4 t = ld_off(p + (size_t)c * S, off);
        v[2 * c] = {t.x, t.y};
        v[2 * c + 1] = {t.z, t.w};
    }
}

__device__ __forceinline__ void store_spinor(double2 *__restrict__ p, int S, int s, const cpx<double> v[12])
{
    const uint32_t off = (uint32_t)s * 16u;
#pragma unroll
    for (int c = 0; c < 12; ++c) st_off(p + (size_t)c * S, off, make_double2(v[c].r, v[c].i));
}

__device__ __forceinline__ void store_spinor(float4 *__restrict__ p, int S, int s, const cpx<float> v[12])
{
    const uint32_t off = (uint32_t)s * 16u;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        st_off(p + (size_t)c * S, off, make_float4(v[2 * c].r, v[2 * c].i, v[2 * c + 1].r, v[2 * c + 1].i));
}

// non-temporal forms (streaming stores that do not keep the lines in L2)
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ void st_off_nt(void *__restrict__ base, uint32_t byte_off, T v)
{
    SGN_GLOBAL char *b = (SGN_GLOBAL char *)base;
    __builtin_nontemporal_store(v, reinterpret_cast<SGN_GLOBAL T *>(b + byte_off));
}

__device__ __forceinline__ void store_spinor_nt(double2 *__restrict__ p, int S, int s, const cpx<double> v[12])
{
    const uint32_t off = (uint32_t)s * 16u;
#pragma unroll
    for (int c = 0; c < 12; ++c) st_off_nt<nt_d2>(p + (size_t)c * S, off, nt_d2{v[c].r, v[c].i});
}

__device__ __forceinline__ void store_spinor_nt(float4 *__restrict__ p, int S, int s, const cpx<float> v[12])
{
    const uint32_t off = (uint32_t)s * 16u;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        st_off_nt<nt_f4>(p + (size_t)c * S, off, nt_f4{v[2 * c].r, v[2 * c].i, v[2 * c + 1].r, v[2 * c + 1].i});
}

// conj(a b - c d), written as one multiply and three fused multiply-adds per
// real component (the compiler does not reassociate the plain expression)
template <typename R>
__device__ __forceinline__ cpx<R> conj_cross(cpx<R> a, cpx<R> b, cpx<R> c, cpx<R> d)
{
    R re = a.r * b.r;
    re = fma(-a.i, b.i, re);
    re = fma(-c.r, d.r, re);
    re = fma(c.i, d.i, re);
    R im = -(a.r * b.i);
    im = fma(-a.i, b.r, im);
    im = fma(c.r, d.i, im);
    im = fma(c.i, d.r, im);
    return {re, im};
}

// Third row of an SU(3) matrix from its first two: u2 = conj(u0 x u1).
template <typename R>
__device__ __forceinline__ void su3_third_row(cpx<R> u[9])
{
    u[6] = conj_cross(u[1], u[5], u[2], u[4]);
    u[7] = conj_cross(u[2], u[3], u[0], u[5]);
    u[8] = conj_cross(u[0], u[4], u[1], u[3]);
}

template <typename R>
__device__ __forceinline__ void link_entry(const double2 *b, uint32_t off, cpx<R> &u)
{
    double2 t = ld_off(b, off * 16u);
    u = {static_cast<R>(t.x), static_cast<R>(t.y)};
}
template <typename R>
__device__ __forceinline__ void link_entry(const float2 *b, uint32_t off, cpx<R> &u)
{
    float2 t = ld_off(b, off * 8u);
    u = {static_cast<R>(t.x), static_cast<R>(t.y)};
}
template <typename R>
__device__ __forceinline__ void link_entry(const __half2 *b, uint32_t off, cpx<R> &u)
{
    float2 t = __half22float2(ld_off(b, off * 4u));
    u = {static_cast<R>(t.x), static_cast<R>(t.y)};
}

// one stored link entry as a complex number of the arithmetic precision
template <typename R> __device__ __forceinline__ cpx<R> to_cpx(double2 v) { return {static_cast<R>(v.x), static_cast<R>(v.y)}; }
template <typename R> __device__ __forceinline__ cpx<R> to_cpx(float2 v) { return {static_cast<R>(v.x), static_cast<R>(v.y)}; }
template <typename R> __device__ __forceinline__ cpx<R> to_cpx(__half2 v)
{
    const float2 t = __half22float2(v);
    return {static_cast<R>(t.x), static_cast<R>(t.y)};
}

// U_nu(x) at site s from the [4][ne][S] link array (ne = 6: two rows stored,
// the third rebuilt; ne = 9: all entries)
template <typename R, typename LT>
__device__ __forceinline__ void load_link(const LT *__restrict__ U, int S, int ne, int nu, int s, cpx<R> u[9])
{
    const LT *b = U + (size_t)nu * ne * S;
    if (ne == 6) {
#pragma unroll
        for (int e = 0; e < 6; ++e) link_entry<R>(b + (size_t)e * S, (uint32_t)s, u[e]);
        su3_third_row(u);
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) link_entry<R>(b + (size_t)e * S, (uint32_t)s, u[e]);
    }
}

// XCD-aware block order: consecutive hardware block ids are dealt round-robin
// to the 8 XCDs, so hardware block i is mapped to a logical block such that
// each XCD walks one contiguous slab of the lattice (t-neighbours then mostly
// hit its own L2).  Bijective on [0, nblk).
__device__ __forceinline__ int xcd_block(int i, int nblk)
{
    constexpr int kXcd = 8;
    int per = nblk / kXcd, rem = nblk % kXcd;
    int k = i % kXcd, j = i / kXcd;
    return k * per + (k < rem ? k : rem) + j;
}

// FP64 sum over a 256-thread block (4 wavefronts of 64); result valid in thread 0.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds /* [(blockDim/64)*NV] */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wid * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += lds[w * NV + k];
            v[k] = s;
        }
    }
}

}  // namespace sgn
