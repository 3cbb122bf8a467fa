// Level-1 vector kernels with deterministic FP64 reductions.
//
// Vectors are flat arrays of complex numbers (the internal spinor layouts are
// flat complex arrays of length 12 V as far as element-wise work is
// concerned).  A reduction is two launches: a producer that writes one
// partial sum per block (grid-stride, at most kMaxBlocks blocks) and a 1-block
// finalize that adds them in block order -- the same result on every run.
#pragma once

#include "sgn_internal.h"

namespace sgn {

constexpr int kVecThreads = 256;
constexpr int kMaxBlocks = 1024;
constexpr int kGramBlocks = 2048;

int vec_blocks(int64_t n);

// partials[b] = sum over the block's elements of conj(x) * y (complex128 / complex64 inputs)
int dot_partials(const void *x, const void *y, int64_t n, bool f32, z64 *partials, hipStream_t s);
// partials[b] = sum |x|^2 (stored in .r)
int norm2_partials(const void *x, int64_t n, bool f32, z64 *partials, hipStream_t s);
// out[0] = sum_b partials[b]   (device)
void finalize_sum(const z64 *partials, int nblk, z64 *out, hipStream_t s);
// blocking FP64 dot (host result) -- setup paths only
z64 dot_sync(Context &ctx, const void *x, const void *y, int64_t n, bool f32, hipStream_t s);
double norm_sync(Context &ctx, const void *x, int64_t n, bool f32, hipStream_t s);

// y = a * x + b * y  (complex128, host scalars)
void axpby64(z64 a, const void *x, z64 b, void *y, int64_t n, hipStream_t s);
// y = a * x  (complex128)
void scale64(z64 a, const void *x, void *y, int64_t n, hipStream_t s);

// precision conversion between the internal FP64 ([12][S] double2) and FP32 ([6][S] float4) spinor
// layouts (S: the lattice's component stride)
void convert_64_to_32(const void *x64, void *x32, int64_t S, hipStream_t s);
void convert_32_to_64(const void *x32, void *x64, int64_t S, hipStream_t s);

// LR deflation on canonical complex128 vectors of length n, with m vectors
// stored back to back (X + i*n):
//   c[i] = X_i^H y                              (deflate_dots, c on device)
//   y = alpha * y + beta * sum_i X_i (d_i c[i])  (deflate_combine; d on device or null = 1)
// f32: X and y hold complex64 entries (the coefficients and sums stay FP64).
void deflate_dots(const void *X, int m, const void *y, int64_t n, z64 *c_dev, Context &ctx, hipStream_t s,
                  bool f32 = false);
// bytes of the context's partials buffer that deflate_dots uses for m vectors of length n
size_t deflate_partials_bytes(int m, int64_t n);
void deflate_combine(void *y, z64 alpha, z64 beta, const void *X, int m, const z64 *c_dev, const z64 *d_dev,
                     int64_t n, hipStream_t s, bool f32 = false);
// out[i] = {||X_i||^2, 0} for the m complex128 vectors X_i (device)
void deflate_norms(const void *X, int m, int64_t n, z64 *out_dev, Context &ctx, hipStream_t s);

// Arnoldi orthogonalisation on a basis X of m vectors (same layout and precision as y):
//   (gram_dots uses up to 2 m kGramBlocks partials)
//   c1[i] = X_i^H y1 and c2[i] = X_i^H y2 in one pass over X  (gram_dots, c on device)
//   y -= sum_i X_i c[i], partials[b] = sum |y|^2 of the new y  (combine_norm; returns the block count,
//   vec_blocks(n), of the partials)
void gram_dots(const void *X, int m, const void *y1, const void *y2, int64_t n, z64 *c1_dev, z64 *c2_dev,
               Context &ctx, hipStream_t s, bool f32);
int combine_norm(void *y, const void *X, int m, const z64 *c_dev, int64_t n, z64 *partials, hipStream_t s, bool f32);

// LR-deflation prologue shared by the solvers (canonical complex128 vectors):
// x = x_P = R sign(Lambda) L^H b, r = (I - R L^H) b and, if rt != nullptr, the
// modified shadow vector rt = (I - L R^H) b.  Null x / r skip that output.
// With check (and r given) the set is first tested for L^H R = I: r holds
// u = R v for a fixed probe v of unit-modulus entries, and every entry of
// L^H u - v must lie within kBiorthTol ||l_i|| ||u|| (SGN_ERR_INVALID otherwise).
// Scratch comes from the context's small device buffer; the stream is
// synchronised when host data is uploaded (x or check), not otherwise.
constexpr double kBiorthTol = 1e-8;
void deflation_prologue(Context &ctx, const sgn_deflation *defl, int64_t n, const void *b, void *x, void *r,
                        void *rt, hipStream_t s, bool check = true);

}  // namespace sgn
