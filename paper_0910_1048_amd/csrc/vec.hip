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
constexpr int kDotBlocks = 2048;  // blocks per pass (grid-stride over the elements; enough loads in flight)

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

// conj(a) . b accumulated in FP64: one complex entry (double2, float2) or two (float4)
__device__ __forceinline__ void acc_cdot(double2 a, double2 b, double &re, double &im)
{
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
}
__device__ __forceinline__ void acc_cdot(float2 a, float2 b, double &re, double &im)
{
    re += (double)a.x * b.x + (double)a.y * b.y;
    im += (double)a.x * b.y - (double)a.y * b.x;
}
__device__ __forceinline__ void acc_cdot(float4 a, float4 b, double &re, double &im)
{
    re += (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
    im += (double)a.x * b.y - (double)a.y * b.x + (double)a.z * b.w - (double)a.w * b.z;
}

// Two right-hand sides in one pass over X: partials[i * gridDim.x + b] for conj(X_i) . y1 and
// partials[(m + i) * gridDim.x + b] for conj(X_i) . y2, the kDotGroup vectors i of group blockIdx.y
// (T = float4 takes complex64 entries two at a time: n counts such pairs)
template <typename T>
__global__ void __launch_bounds__(256) mdot2_kernel(const T *X, const T *y1, const T *y2, int64_t n, int m,
                                                    z64 *partials)
{
    const int i0 = blockIdx.y * kDotGroup;
    const int cnt = min(kDotGroup, m - i0);
    double acc[4 * kDotGroup];
#pragma unroll
    for (int c = 0; c < 4 * kDotGroup; ++c) acc[c] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const T b1 = y1[e], b2 = y2[e];
#pragma unroll
        for (int c = 0; c < kDotGroup; ++c) {
            if (c < cnt) {
                const T a = X[(int64_t)(i0 + c) * n + e];
                acc_cdot(a, b1, acc[2 * c], acc[2 * c + 1]);
                acc_cdot(a, b2, acc[2 * kDotGroup + 2 * c], acc[2 * kDotGroup + 2 * c + 1]);
            }
        }
    }
    __shared__ double lds[4 * kDotGroup * 4];
    block_sum<4 * kDotGroup>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < kDotGroup; ++c) {  // constant indices keep acc in registers
            if (c < cnt) {
                partials[(int64_t)(i0 + c) * gridDim.x + blockIdx.x] = {acc[2 * c], acc[2 * c + 1]};
                partials[(int64_t)(m + i0 + c) * gridDim.x + blockIdx.x] = {acc[2 * kDotGroup + 2 * c],
                                                                             acc[2 * kDotGroup + 2 * c + 1]};
            }
        }
    }
}

// grid (nbx, m): partials[i * nbx + bx] = {sum |X_i|^2 over the block's slice, 0}
template <typename T>
__global__ void __launch_bounds__(256) mnorm_kernel(const T *X, int64_t n, z64 *partials)
{
    const int i = blockIdx.y;
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const T a = X[(int64_t)i * n + e];
        acc[0] += (double)a.x * a.x + (double)a.y * a.y;
    }
    __shared__ double lds[4];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partials[(int64_t)i * gridDim.x + blockIdx.x] = {acc[0], 0.0};
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
        int i = 0;
        for (; i + 4 <= m; i += 4) {  // four independent loads in flight
            T xv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[q] = X[(int64_t)(i + q) * n + e];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                z64 ci = c[i + q];
                if (d) ci = d[i + q] * ci;
                acc = acc + z64{(double)xv[q].x, (double)xv[q].y} * ci;
            }
        }
        for (; i < m; ++i) {
            z64 ci = c[i];
            if (d) ci = d[i] * ci;
            const T xv = X[(int64_t)i * n + e];
            acc = acc + z64{(double)xv.x, (double)xv.y} * ci;
        }
        z64 r = beta * acc;
        if (alpha.r != 0.0 || alpha.i != 0.0) {  // alpha = 0: y is write-only (it may hold anything)
            const T yv = y[e];
            r = r + alpha * z64{(double)yv.x, (double)yv.y};
        }
        y[e] = mk2<T>(r.r, r.i);
    }
}

// y -= sum_i X_i c[i]; partials[block] = sum |y|^2 of the stored (rounded) new y over the block's slice
template <typename T>
__global__ void __launch_bounds__(256) mcombine_norm_kernel(T *y, const T *X, int m, const z64 *c, int64_t n,
                                                            z64 *partials)
{
    double nrm = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        z64 acc = {0.0, 0.0};
        int i = 0;
        for (; i + 4 <= m; i += 4) {  // four independent loads in flight
            const T x0 = X[(int64_t)i * n + e], x1 = X[(int64_t)(i + 1) * n + e], x2 = X[(int64_t)(i + 2) * n + e],
                    x3 = X[(int64_t)(i + 3) * n + e];
            acc = acc + z64{(double)x0.x, (double)x0.y} * c[i];
            acc = acc + z64{(double)x1.x, (double)x1.y} * c[i + 1];
            acc = acc + z64{(double)x2.x, (double)x2.y} * c[i + 2];
            acc = acc + z64{(double)x3.x, (double)x3.y} * c[i + 3];
        }
        for (; i < m; ++i) {
            const T xv = X[(int64_t)i * n + e];
            acc = acc + z64{(double)xv.x, (double)xv.y} * c[i];
        }
        const T yv = y[e];
        const T r = mk2<T>((double)yv.x - acc.r, (double)yv.y - acc.i);
        y[e] = r;
        nrm += (double)r.x * r.x + (double)r.y * r.y;
    }
    __shared__ double lds[4];
    double v[1] = {nrm};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = {v[0], 0.0};
}

// mcombine_norm_kernel for complex64 vectors taken two entries at a time (n2 float4 pairs)
__global__ void __launch_bounds__(256) mcombine_norm_pairs_kernel(float4 *y, const float4 *X, int m, const z64 *c,
                                                                  int64_t n2, z64 *partials)
{
    double nrm = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += (int64_t)gridDim.x * blockDim.x) {
        z64 a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
        int i = 0;
        for (; i + 4 <= m; i += 4) {
            float4 xv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[q] = X[(int64_t)(i + q) * n2 + e];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a0 = a0 + z64{(double)xv[q].x, (double)xv[q].y} * c[i + q];
                a1 = a1 + z64{(double)xv[q].z, (double)xv[q].w} * c[i + q];
            }
        }
        for (; i < m; ++i) {
            const float4 xv = X[(int64_t)i * n2 + e];
            a0 = a0 + z64{(double)xv.x, (double)xv.y} * c[i];
            a1 = a1 + z64{(double)xv.z, (double)xv.w} * c[i];
        }
        const float4 yv = y[e];
        const float4 r = make_float4((float)((double)yv.x - a0.r), (float)((double)yv.y - a0.i),
                                     (float)((double)yv.z - a1.r), (float)((double)yv.w - a1.i));
        y[e] = r;
        nrm += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z + (double)r.w * r.w;
    }
    __shared__ double lds[4];
    double v[1] = {nrm};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = {v[0], 0.0};
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

size_t deflate_partials_bytes(int m, int64_t n)
{
    const int nbx = std::max(1, std::min(kDotBlocks, (int)((n + 255) / 256)));
    return (size_t)std::max(m, 0) * nbx * sizeof(z64);
}

void deflate_dots(const void *X, int m, const void *y, int64_t n, z64 *c_dev, Context &ctx, hipStream_t s, bool f32)
{
    if (m <= 0) return;
    const int nbx = std::max(1, std::min(kDotBlocks, (int)((n + 255) / 256)));
    const int ng = (m + kDotGroup - 1) / kDotGroup;
    z64 *part = static_cast<z64 *>(ctx.ensure_partials(deflate_partials_bytes(m, n)));
    if (f32)
        hipLaunchKernelGGL(mdot_kernel<float2>, dim3(nbx, ng), dim3(256), 0, s, (const float2 *)X, (const float2 *)y, n,
                           m, part);
    else
        hipLaunchKernelGGL(mdot_kernel<double2>, dim3(nbx, ng), dim3(256), 0, s, (const double2 *)X, (const double2 *)y,
                           n, m, part);
    hipLaunchKernelGGL(mfinalize_kernel, dim3(m), dim3(256), 0, s, part, nbx, c_dev);
    SGN_HIP(hipGetLastError());
}

void deflate_norms(const void *X, int m, int64_t n, z64 *out_dev, Context &ctx, hipStream_t s)
{
    if (m <= 0) return;
    const int nbx = std::max(1, std::min(kDotBlocks, (int)((n + 255) / 256)));
    z64 *part = static_cast<z64 *>(ctx.ensure_partials((size_t)m * nbx * sizeof(z64)));
    hipLaunchKernelGGL(mnorm_kernel<double2>, dim3(nbx, m), dim3(256), 0, s, (const double2 *)X, n, part);
    hipLaunchKernelGGL(mfinalize_kernel, dim3(m), dim3(256), 0, s, part, nbx, out_dev);
    SGN_HIP(hipGetLastError());
}

void gram_dots(const void *X, int m, const void *y1, const void *y2, int64_t n, z64 *c1_dev, z64 *c2_dev,
               Context &ctx, hipStream_t s, bool f32)
{
    if (m <= 0) return;
    // enough blocks to keep loads in flight when there is a single group (small m)
    const int nbx = std::max(1, std::min(kGramBlocks, (int)((n + 255) / 256)));
    const int ng = (m + kDotGroup - 1) / kDotGroup;
    z64 *part = static_cast<z64 *>(ctx.ensure_partials((size_t)2 * m * nbx * sizeof(z64)));
    if (f32 && n % 2 == 0)  // pairs of complex64 entries: 16-byte loads, as for complex128
        hipLaunchKernelGGL(mdot2_kernel<float4>, dim3(nbx, ng), dim3(256), 0, s, (const float4 *)X, (const float4 *)y1,
                           (const float4 *)y2, n / 2, m, part);
    else if (f32)
        hipLaunchKernelGGL(mdot2_kernel<float2>, dim3(nbx, ng), dim3(256), 0, s, (const float2 *)X, (const float2 *)y1,
                           (const float2 *)y2, n, m, part);
    else
        hipLaunchKernelGGL(mdot2_kernel<double2>, dim3(nbx, ng), dim3(256), 0, s, (const double2 *)X,
                           (const double2 *)y1, (const double2 *)y2, n, m, part);
    hipLaunchKernelGGL(mfinalize_kernel, dim3(m), dim3(256), 0, s, part, nbx, c1_dev);
    hipLaunchKernelGGL(mfinalize_kernel, dim3(m), dim3(256), 0, s, part + (size_t)m * nbx, nbx, c2_dev);
    SGN_HIP(hipGetLastError());
}

int combine_norm(void *y, const void *X, int m, const z64 *c_dev, int64_t n, z64 *partials, hipStream_t s, bool f32)
{
    const int nb = vec_blocks(n);
    if (f32 && n % 2 == 0)
        hipLaunchKernelGGL(mcombine_norm_pairs_kernel, dim3(nb), dim3(256), 0, s, (float4 *)y, (const float4 *)X, m,
                           c_dev, n / 2, partials);
    else if (f32)
        hipLaunchKernelGGL(mcombine_norm_kernel<float2>, dim3(nb), dim3(256), 0, s, (float2 *)y, (const float2 *)X, m,
                           c_dev, n, partials);
    else
        hipLaunchKernelGGL(mcombine_norm_kernel<double2>, dim3(nb), dim3(256), 0, s, (double2 *)y,
                           (const double2 *)X, m, c_dev, n, partials);
    SGN_HIP(hipGetLastError());
    return nb;
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
