// Level-1 vector kernels, deterministic FP64 reductions, precision conversion
// and the LR-deflation projections.  All of these are HBM-bound streaming
// kernels: grid-stride loops over at most kMaxBlocks blocks of 256 threads.
#include "vec.h"

#include "field_io.h"

namespace sgn {

int vec_blocks(int64_t n)
{
    int64_t b = (n + kVecThreads - 1) / kVecThreads;
    if (b < 1) b = 1;
    return (int)(b < kMaxBlocks ? b : kMaxBlocks);
}

namespace {

__device__ __forceinline__ z64 ld64(const void *p, int64_t i)
{
    double2 t = static_cast<const double2 *>(p)[i];
    return {t.x, t.y};
}

__device__ __forceinline__ z64 ld32(const void *p, int64_t i)
{
    float2 t = static_cast<const float2 *>(p)[i];
    return {(double)t.x, (double)t.y};
}

template <bool F32>
__global__ void __launch_bounds__(256) dot_kernel(const void *x, const void *y, int64_t n, z64 *partials)
{
    double re = 0.0, im = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        z64 a = F32 ? ld32(x, i) : ld64(x, i);
        z64 b = F32 ? ld32(y, i) : ld64(y, i);
        re += a.r * b.r + a.i * b.i;
        im += a.r * b.i - a.i * b.r;
    }
    __shared__ double lds[8];
    double v[2] = {re, im};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = {v[0], v[1]};
}

template <bool F32>
__global__ void __launch_bounds__(256) norm2_kernel(const void *x, int64_t n, z64 *partials)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        z64 a = F32 ? ld32(x, i) : ld64(x, i);
        acc += a.r * a.r + a.i * a.i;
    }
    __shared__ double lds[4];
    double v[1] = {acc};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = {v[0], 0.0};
}

// sum partials in block order (one block; threads take strided slices, then a fixed-order combine)
__global__ void __launch_bounds__(256) finalize_kernel(const z64 *partials, int nblk, z64 *out)
{
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        re += partials[i].r;
        im += partials[i].i;
    }
    __shared__ double lds[8];
    double v[2] = {re, im};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) *out = {v[0], v[1]};
}

__global__ void axpby64_kernel(z64 a, const double2 *x, z64 b, double2 *y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double2 xv = x[i], yv = y[i];
        z64 r = a * z64{xv.x, xv.y} + b * z64{yv.x, yv.y};
        y[i] = make_double2(r.r, r.i);
    }
}

__global__ void scale64_kernel(z64 a, const double2 *x, double2 *y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double2 xv = x[i];
        z64 r = a * z64{xv.x, xv.y};
        y[i] = make_double2(r.r, r.i);
    }
}

__global__ void cvt64to32(const double2 *__restrict__ x, float4 *__restrict__ y, int S)
{
    const int64_t n = (int64_t)6 * S;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(p / S), s = (int)(p - (int64_t)c2 * S);
        double2 a = x[(int64_t)(2 * c2) * S + s], b = x[(int64_t)(2 * c2 + 1) * S + s];
        y[p] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
    }
}

__global__ void cvt32to64(const float4 *__restrict__ x, double2 *__restrict__ y, int S)
{
    const int64_t n = (int64_t)6 * S;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int c2 = (int)(p / S), s = (int)(p - (int64_t)c2 * S);
        float4 t = x[p];
        y[(int64_t)(2 * c2) * S + s] = make_double2(t.x, t.y);
        y[(int64_t)(2 * c2 + 1) * S + s] = make_double2(t.z, t.w);
    }
}

// grid (nbx, m): partials[i * nbx + bx] = sum conj(X_i) y over the block's slice
// (T = double2 or float2; FP64 accumulation either way)
constexpr int kDotGroup = 8;   // dot products per pass of y
constexpr int kDotBlocks = 512;  // blocks per pass (grid-stride over the elements)

// partials[i * gridDim.x + b] = sum over block b's slice of conj(X_i) . y for the kDotGroup
// vectors i of group blockIdx.y (fewer in the last group); y is read once per group
template <typename T>
__global__ void __launch_bounds__(256) mdot_kernel(const T *X, const T *y, int64_t n, int m, z64 *partials)
{
    const int i0 = blockIdx.y * kDotGroup;
    const int cnt = min(kDotGroup, m - i0);
    double acc[2 * kDotGroup];
#pragma unroll
    for (int c = 0; c < 2 * kDotGroup; ++c) acc[c] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const T b = y[e];
#pragma unroll
        for (int c = 0; c < kDotGroup; ++c) {
            if (c < cnt) {
                const T a = X[(int64_t)(i0 + c) * n + e];
                acc[2 * c] += (double)a.x * b.x + (double)a.y * b.y;
                acc[2 * c + 1] += (double)a.x * b.y - (double)a.y * b.x;
            }
        }
    }
    __shared__ double lds[2 * kDotGroup * 4];
    block_sum<2 * kDotGroup>(acc, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < cnt; ++c) partials[(int64_t)(i0 + c) * gridDim.x + blockIdx.x] = {acc[2 * c], acc[2 * c + 1]};
}

__global__ void __launch_bounds__(256) mfinalize_kernel(const z64 *partials, int nbx, z64 *out)
{
    const int i = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < nbx; b += blockDim.x) {
        re += partials[(int64_t)i * nbx + b].r;
        im += partials[(int64_t)i * nbx + b].i;
    }
    __shared__ double lds[8];
    double v[2] = {re, im};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) out[i] = {v[0], v[1]};
}

template <typename T>
__device__ __forceinline__ T mk2(double a, double b);
template <> __device__ __forceinline__ double2 mk2<double2>(double a, double b) { return make_double2(a, b); }
template <> __device__ __forceinline__ float2 mk2<float2>(double a, double b) { return make_float2((float)a, (float)b); }

template <typename T>
__global__ void mcombine_kernel(T *y, z64 alpha, z64 beta, const T *X, int m, const z64 *c, const z64 *d, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        z64 acc = {0.0, 0.0};
        for (int i = 0; i < m; ++i) {
            z64 ci = c[i];
            if (d) ci = d[i] * ci;
            const T xv = X[(int64_t)i * n + e];
            acc = acc + z64{(double)xv.x, (double)xv.y} * ci;
        }
        const T yv = y[e];
        z64 r = alpha * z64{(double)yv.x, (double)yv.y} + beta * acc;
        y[e] = mk2<T>(r.r, r.i);
    }
}

// partials[block] = ( sum |y - x|^2 , sum |x|^2 ) over the block's slice
__global__ void __launch_bounds__(256) diff_norm_kernel(const double2 *x, const double2 *y, int64_t n, z64 *partials)
{
    double d = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double2 a = x[i], c = y[i];
        const double er = c.x - a.x, ei = c.y - a.y;
        d += er * er + ei * ei;
        b += a.x * a.x + a.y * a.y;
    }
    __shared__ double lds[8];
    double v[2] = {d, b};
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = {v[0], v[1]};
}

}  // namespace

int dot_partials(const void *x, const void *y, int64_t n, bool f32, z64 *partials, hipStream_t s)
{
    const int nb = vec_blocks(n);
    if (f32)
        hipLaunchKernelGGL(dot_kernel<true>, dim3(nb), dim3(256), 0, s, x, y, n, partials);
    else
        hipLaunchKernelGGL(dot_kernel<false>, dim3(nb), dim3(256), 0, s, x, y, n, partials);
    SGN_HIP(hipGetLastError());
    return nb;
}

int norm2_partials(const void *x, int64_t n, bool f32, z64 *partials, hipStream_t s)
{
    const int nb = vec_blocks(n);
    if (f32)
        hipLaunchKernelGGL(norm2_kernel<true>, dim3(nb), dim3(256), 0, s, x, n, partials);
    else
        hipLaunchKernelGGL(norm2_kernel<false>, dim3(nb), dim3(256), 0, s, x, n, partials);
    SGN_HIP(hipGetLastError());
    return nb;
}

void finalize_sum(const z64 *partials, int nblk, z64 *out, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, partials, nblk, out);
    SGN_HIP(hipGetLastError());
}

z64 dot_sync(Context &ctx, const void *x, const void *y, int64_t n, bool f32, hipStream_t s)
{
    z64 *part = static_cast<z64 *>(ctx.ensure_partials((kMaxBlocks + 1) * sizeof(z64)));
    const int nb = dot_partials(x, y, n, f32, part, s);
    finalize_sum(part, nb, part + kMaxBlocks, s);
    z64 h;
    SGN_HIP(hipMemcpyAsync(&h, part + kMaxBlocks, sizeof(z64), hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    return h;
}

double norm_sync(Context &ctx, const void *x, int64_t n, bool f32, hipStream_t s)
{
    z64 *part = static_cast<z64 *>(ctx.ensure_partials((kMaxBlocks + 1) * sizeof(z64)));
    const int nb = norm2_partials(x, n, f32, part, s);
    finalize_sum(part, nb, part + kMaxBlocks, s);
    z64 h;
    SGN_HIP(hipMemcpyAsync(&h, part + kMaxBlocks, sizeof(z64), hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    return std::sqrt(h.r);
}

void axpby64(z64 a, const void *x, z64 b, void *y, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(axpby64_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, a, (const double2 *)x, b,
                       (double2 *)y, n);
    SGN_HIP(hipGetLastError());
}

void scale64(z64 a, const void *x, void *y, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(scale64_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, a, (const double2 *)x,
                       (double2 *)y, n);
    SGN_HIP(hipGetLastError());
}

void convert_64_to_32(const void *x64, void *x32, int64_t S, hipStream_t s)
{
    hipLaunchKernelGGL(cvt64to32, dim3(vec_blocks(6 * S)), dim3(256), 0, s, (const double2 *)x64, (float4 *)x32,
                       (int)S);
    SGN_HIP(hipGetLastError());
}

void convert_32_to_64(const void *x32, void *x64, int64_t S, hipStream_t s)
{
    hipLaunchKernelGGL(cvt32to64, dim3(vec_blocks(6 * S)), dim3(256), 0, s, (const float4 *)x32, (double2 *)x64,
                       (int)S);
    SGN_HIP(hipGetLastError());
}

void deflate_dots(const void *X, int m, const void *y, int64_t n, z64 *c_dev, Context &ctx, hipStream_t s, bool f32)
{
    if (m <= 0) return;
    const int nbx = std::max(1, std::min(kDotBlocks, vec_blocks(n)));
    const int ng = (m + kDotGroup - 1) / kDotGroup;
    z64 *part = static_cast<z64 *>(ctx.ensure_partials((size_t)m * nbx * sizeof(z64)));
    if (f32)
        hipLaunchKernelGGL(mdot_kernel<float2>, dim3(nbx, ng), dim3(256), 0, s, (const float2 *)X, (const float2 *)y, n,
                           m, part);
    else
        hipLaunchKernelGGL(mdot_kernel<double2>, dim3(nbx, ng), dim3(256), 0, s, (const double2 *)X, (const double2 *)y,
                           n, m, part);
    hipLaunchKernelGGL(mfinalize_kernel, dim3(m), dim3(256), 0, s, part, nbx, c_dev);
    SGN_HIP(hipGetLastError());
}

void deflate_combine(void *y, z64 alpha, z64 beta, const void *X, int m, const z64 *c_dev, const z64 *d_dev,
                     int64_t n, hipStream_t s, bool f32)
{
    if (f32)
        hipLaunchKernelGGL(mcombine_kernel<float2>, dim3(vec_blocks(n)), dim3(256), 0, s, (float2 *)y, alpha, beta,
                           (const float2 *)X, m, c_dev, d_dev, n);
    else
        hipLaunchKernelGGL(mcombine_kernel<double2>, dim3(vec_blocks(n)), dim3(256), 0, s, (double2 *)y, alpha, beta,
                           (const double2 *)X, m, c_dev, d_dev, n);
    SGN_HIP(hipGetLastError());
}

}  // namespace sgn

extern "C" sgn_status sgn_accuracy_measure(sgn_lattice l, const void *b, const void *ssb, double *acc, void *stream)
{
    using namespace sgn;
    return guard([&] {
        SGN_REQUIRE(l && b && ssb && acc, "sgn_accuracy_measure: null argument");
        Lattice &lat = *as_lattice(l);
        SGN_HIP(hipSetDevice(lat.ctx->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int64_t n = 12 * lat.V;
        z64 *part = static_cast<z64 *>(lat.ctx->ensure_partials((kMaxBlocks + 1) * sizeof(z64)));
        const int nb = vec_blocks(n);
        hipLaunchKernelGGL(diff_norm_kernel, dim3(nb), dim3(256), 0, s, (const double2 *)b, (const double2 *)ssb,
                           n, part);
        SGN_HIP(hipGetLastError());
        finalize_sum(part, nb, part + kMaxBlocks, s);
        z64 h;
        SGN_HIP(hipMemcpyAsync(&h, part + kMaxBlocks, sizeof(z64), hipMemcpyDeviceToHost, s));
        SGN_HIP(hipStreamSynchronize(s));
        SGN_REQUIRE(h.i > 0.0, "sgn_accuracy_measure: b is zero");
        *acc = 0.5 * std::sqrt(h.r / h.i);
    });
}
