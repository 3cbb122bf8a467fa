// Context, lattice objects, layout conversion and status strings.
#include "field_io.h"

#include <cmath>
#include <cstring>
#include <mutex>

namespace sgn {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

void *Context::ensure_partials(size_t bytes)
{
    if (bytes > partials_bytes) {
        SGN_HIP(hipDeviceSynchronize());  // kernels of earlier calls may still use the old buffer
        if (partials) SGN_HIP(hipFree(partials));
        partials = nullptr;
        partials_bytes = 0;
        if (hipMalloc(&partials, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "partials buffer"};
        partials_bytes = bytes;
    }
    return partials;
}

void *Context::ensure_scalars(size_t bytes)
{
    if (bytes > scalars_bytes) {
        SGN_HIP(hipDeviceSynchronize());
        if (scalars) SGN_HIP(hipFree(scalars));
        scalars = nullptr;
        scalars_bytes = 0;
        if (hipMalloc(&scalars, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "scalar buffer"};
        scalars_bytes = bytes;
    }
    return scalars;
}

void *Context::ensure_arena(size_t bytes)
{
    if (bytes > arena_bytes) {
        SGN_HIP(hipDeviceSynchronize());
        if (arena) SGN_HIP(hipFree(arena));
        arena = nullptr;
        arena_bytes = 0;
        if (hipMalloc(&arena, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "solver workspace"};
        // padding entries of internal fields must read as zero in every reduction;
        // kernels never write non-zero values there, so clearing once suffices
        SGN_HIP(hipMemset(arena, 0, bytes));
        arena_bytes = bytes;
    }
    return arena;
}

void *Context::ensure_small(size_t bytes)
{
    if (bytes > small_bytes) {
        SGN_HIP(hipDeviceSynchronize());
        if (small) SGN_HIP(hipFree(small));
        small = nullptr;
        small_bytes = 0;
        bytes = std::max<size_t>(bytes, 4096);
        if (hipMalloc(&small, bytes) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "deflation scratch"};
        small_bytes = bytes;
    }
    return small;
}

void Lattice::ensure_stage(size_t bytes)
{
    if (bytes <= stage_bytes) return;
    SGN_HIP(hipDeviceSynchronize());
    if (stage_in) SGN_HIP(hipFree(stage_in));
    if (stage_out) SGN_HIP(hipFree(stage_out));
    stage_in = stage_out = nullptr;
    stage_bytes = 0;
    if (hipMalloc(&stage_in, bytes) != hipSuccess || hipMalloc(&stage_out, bytes) != hipSuccess)
        throw Failure{SGN_ERR_NOMEM, "staging buffers"};
    stage_bytes = bytes;
}

namespace {

// canonical [site][nu][3][3] complex128  ->  [nu][9][V] of LT
template <typename LT> __device__ inline LT to_link(double2 v);
template <> __device__ inline double2 to_link<double2>(double2 v) { return v; }
template <> __device__ inline float2 to_link<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ inline __half2 to_link<__half2>(double2 v)
{
    return __floats2half2_rn((float)v.x, (float)v.y);
}

template <typename LT>
__global__ void pack_links_kernel(const double2 *__restrict__ canon, LT *__restrict__ out, int V, int S, int ne)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * V) return;
    const int s = t / 4, nu = t % 4;
    for (int e = 0; e < ne; ++e) out[((size_t)nu * ne + e) * S + s] = to_link<LT>(canon[(size_t)t * 9 + e]);
}

// Per block: the largest deviation of a link from SU(3), max(|U U^H - I|_ij, |det U - 1|)
__global__ void __launch_bounds__(256) su3_check_kernel(const double2 *__restrict__ canon, int nlinks, double *blockmax)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double dev = 0.0;
    if (t < nlinks) {
        z64 u[9];
        for (int e = 0; e < 9; ++e) {
            const double2 v = canon[(size_t)t * 9 + e];
            u[e] = {v.x, v.y};
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                z64 acc = {i == j ? -1.0 : 0.0, 0.0};
                for (int k = 0; k < 3; ++k) acc = acc + u[3 * i + k] * conj(u[3 * j + k]);
                dev = fmax(dev, sqrt(norm2(acc)));
            }
        const z64 det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                        u[2] * (u[3] * u[7] - u[4] * u[6]);
        dev = fmax(dev, sqrt(norm2(det - z64{1.0, 0.0})));
        if (!(dev == dev)) dev = INFINITY;  // NaN entries: not SU(3)
    }
    __shared__ double red[256];
    red[threadIdx.x] = dev;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}

// internal layouts: padding sites (V <= s < S) are written as zeros
__global__ void pack64(const double2 *__restrict__ c, double2 *__restrict__ o, int V, int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
#pragma unroll
    for (int k = 0; k < 12; ++k) o[(size_t)k * S + s] = s < V ? c[(size_t)s * 12 + k] : make_double2(0.0, 0.0);
}

__global__ void unpack64(const double2 *__restrict__ o, double2 *__restrict__ c, int V, int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int k = 0; k < 12; ++k) c[(size_t)s * 12 + k] = o[(size_t)k * S + s];
}

__global__ void pack32(const float2 *__restrict__ c, float4 *__restrict__ o, int V, int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (s >= V) {
            o[(size_t)k * S + s] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        float2 a = c[(size_t)s * 12 + 2 * k], b = c[(size_t)s * 12 + 2 * k + 1];
        o[(size_t)k * S + s] = make_float4(a.x, a.y, b.x, b.y);
    }
}

__global__ void unpack32(const float4 *__restrict__ o, float2 *__restrict__ c, int V, int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float4 t = o[(size_t)k * S + s];
        c[(size_t)s * 12 + 2 * k] = make_float2(t.x, t.y);
        c[(size_t)s * 12 + 2 * k + 1] = make_float2(t.z, t.w);
    }
}

// ---------------------------------------------------------------- temporal gauge
// A site-local colour rotation G(x) in SU(3) maps the field to U'_nu(x) = G(x) U_nu(x) G(x + nu)^H and
// a spinor to psi'(x) = G(x) psi(x); the operator becomes G D_W G^H (the hops are covariant, gamma5
// and the weights act on spin only), so sign(H'_W) = G sign(H_W) G^H.  With G(x, 0) = 1 and
// G(x, t + 1) = G(x, t) U_t(x, t) along each time line every time link off the last slice is the unit
// matrix, which the stencil then neither loads nor multiplies; the last slice keeps the ordered
// product of the line's time links.

__device__ inline z64 ldc(const double2 *p) { const double2 v = *p; return {v.x, v.y}; }
__device__ inline void stc(double2 *p, z64 v) { *p = make_double2(v.r, v.i); }

// G[s][3][3] (row-major, complex128) for every site; one thread walks one time line
__global__ void tg_gauge_kernel(const double2 *__restrict__ canon, double2 *__restrict__ G, int vs, int lt)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= vs) return;
    z64 g[9];
    for (int e = 0; e < 9; ++e) g[e] = {e % 4 == 0 ? 1.0 : 0.0, 0.0};
    for (int t = 0; t < lt; ++t) {
        const size_t s = (size_t)t * vs + x;
        for (int e = 0; e < 9; ++e) stc(G + s * 9 + e, g[e]);
        if (t + 1 == lt) break;
        z64 u[9], h[9];
        for (int e = 0; e < 9; ++e) u[e] = ldc(canon + (s * 4 + 3) * 9 + e);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                z64 acc = {0.0, 0.0};
                for (int k = 0; k < 3; ++k) acc = acc + g[3 * i + k] * u[3 * k + j];
                h[3 * i + j] = acc;
            }
        for (int e = 0; e < 9; ++e) g[e] = h[e];
    }
}

// U'_nu(x) = G(x) U_nu(x) G(x + nu)^H in the canonical layout; time links off the last slice are
// written as the exact unit matrix
__global__ void tg_links_kernel(const double2 *__restrict__ canon, const double2 *__restrict__ G,
                                double2 *__restrict__ out, int V, int L0, int L1, int L2, int L3)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * V) return;
    const int s = t / 4, nu = t % 4;
    const int L[4] = {L0, L1, L2, L3}, st[4] = {1, L0, L0 * L1, L0 * L1 * L2};
    const int c[4] = {s % L0, (s / L0) % L1, (s / (L0 * L1)) % L2, s / (L0 * L1 * L2)};
    double2 *o = out + (size_t)t * 9;
    if (nu == 3 && c[3] < L3 - 1) {
        for (int e = 0; e < 9; ++e) stc(o + e, {e % 4 == 0 ? 1.0 : 0.0, 0.0});
        return;
    }
    const int n = c[nu] == L[nu] - 1 ? s - (L[nu] - 1) * st[nu] : s + st[nu];
    z64 a[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            z64 acc = {0.0, 0.0};
            for (int k = 0; k < 3; ++k) acc = acc + ldc(G + (size_t)s * 9 + 3 * i + k) * ldc(canon + (size_t)t * 9 + 3 * k + j);
            a[3 * i + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            z64 acc = {0.0, 0.0};
            for (int k = 0; k < 3; ++k) acc = acc + a[3 * i + k] * conj(ldc(G + (size_t)n * 9 + 3 * j + k));
            stc(o + 3 * i + j, acc);
        }
}

// spinor components (spin 4 x colour 3) rotated in colour: G psi (kAdj false) or G^H psi
template <bool kAdj>
__device__ inline void rotate12(const double2 *__restrict__ G, int s, z64 v[12])
{
    z64 g[9];
    for (int e = 0; e < 9; ++e) g[e] = ldc(G + (size_t)s * 9 + e);
    for (int sp = 0; sp < 4; ++sp) {
        const z64 a0 = v[3 * sp], a1 = v[3 * sp + 1], a2 = v[3 * sp + 2];
        for (int i = 0; i < 3; ++i)
            v[3 * sp + i] = kAdj ? cmulc(g[i], a0) + cmulc(g[3 + i], a1) + cmulc(g[6 + i], a2)
                                 : g[3 * i] * a0 + g[3 * i + 1] * a1 + g[3 * i + 2] * a2;
    }
}

// the internal layouts of a temporal-gauge lattice hold G psi; the rotation is done in FP64
__global__ void pack64g(const double2 *__restrict__ c, const double2 *__restrict__ G, double2 *__restrict__ o, int V,
                        int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    z64 v[12];
    for (int k = 0; k < 12; ++k) v[k] = s < V ? ldc(c + (size_t)s * 12 + k) : z64{0.0, 0.0};
    if (s < V) rotate12<false>(G, s, v);
    for (int k = 0; k < 12; ++k) stc(o + (size_t)k * S + s, v[k]);
}

__global__ void unpack64g(const double2 *__restrict__ o, const double2 *__restrict__ G, double2 *__restrict__ c, int V,
                          int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    z64 v[12];
    for (int k = 0; k < 12; ++k) v[k] = ldc(o + (size_t)k * S + s);
    rotate12<true>(G, s, v);
    for (int k = 0; k < 12; ++k) stc(c + (size_t)s * 12 + k, v[k]);
}

__global__ void pack32g(const float2 *__restrict__ c, const double2 *__restrict__ G, float4 *__restrict__ o, int V,
                        int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    z64 v[12];
    for (int k = 0; k < 12; ++k) {
        const float2 a = s < V ? c[(size_t)s * 12 + k] : make_float2(0.f, 0.f);
        v[k] = {(double)a.x, (double)a.y};
    }
    if (s < V) rotate12<false>(G, s, v);
    for (int k = 0; k < 6; ++k)
        o[(size_t)k * S + s] = make_float4((float)v[2 * k].r, (float)v[2 * k].i, (float)v[2 * k + 1].r,
                                           (float)v[2 * k + 1].i);
}

__global__ void unpack32g(const float4 *__restrict__ o, const double2 *__restrict__ G, float2 *__restrict__ c, int V,
                          int S)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    z64 v[12];
    for (int k = 0; k < 6; ++k) {
        const float4 t = o[(size_t)k * S + s];
        v[2 * k] = {(double)t.x, (double)t.y};
        v[2 * k + 1] = {(double)t.z, (double)t.w};
    }
    rotate12<true>(G, s, v);
    for (int k = 0; k < 12; ++k) c[(size_t)s * 12 + k] = make_float2((float)v[k].r, (float)v[k].i);
}

}  // namespace

void pack_spinor(const Lattice &lat, const void *canon, void *internal, sgn_prec p, hipStream_t s)
{
    const int V = (int)lat.V, S = (int)lat.S;
    dim3 g((S + 255) / 256), b(256);
    const double2 *G = static_cast<const double2 *>(lat.gauge);
    if (p == SGN_PREC_F64 && G)
        hipLaunchKernelGGL(pack64g, g, b, 0, s, (const double2 *)canon, G, (double2 *)internal, V, S);
    else if (G)
        hipLaunchKernelGGL(pack32g, g, b, 0, s, (const float2 *)canon, G, (float4 *)internal, V, S);
    else if (p == SGN_PREC_F64)
        hipLaunchKernelGGL(pack64, g, b, 0, s, (const double2 *)canon, (double2 *)internal, V, S);
    else
        hipLaunchKernelGGL(pack32, g, b, 0, s, (const float2 *)canon, (float4 *)internal, V, S);
    SGN_HIP(hipGetLastError());
}

void unpack_spinor(const Lattice &lat, const void *internal, void *canon, sgn_prec p, hipStream_t s)
{
    const int V = (int)lat.V, S = (int)lat.S;
    dim3 g((V + 255) / 256), b(256);
    const double2 *G = static_cast<const double2 *>(lat.gauge);
    if (p == SGN_PREC_F64 && G)
        hipLaunchKernelGGL(unpack64g, g, b, 0, s, (const double2 *)internal, G, (double2 *)canon, V, S);
    else if (G)
        hipLaunchKernelGGL(unpack32g, g, b, 0, s, (const float4 *)internal, G, (float2 *)canon, V, S);
    else if (p == SGN_PREC_F64)
        hipLaunchKernelGGL(unpack64, g, b, 0, s, (const double2 *)internal, (double2 *)canon, V, S);
    else
        hipLaunchKernelGGL(unpack32, g, b, 0, s, (const float4 *)internal, (float2 *)canon, V, S);
    SGN_HIP(hipGetLastError());
}

}  // namespace sgn

using namespace sgn;

extern "C" const char *sgn_status_string(sgn_status s)
{
    switch (s) {
    case SGN_OK: return "ok";
    case SGN_ERR_INVALID: return "invalid argument";
    case SGN_ERR_HIP: return "HIP runtime error";
    case SGN_ERR_NOMEM: return "out of device memory";
    case SGN_ERR_BREAKDOWN: return "Krylov breakdown";
    case SGN_ERR_NOT_CONVERGED: return "not converged";
    case SGN_ERR_IMAG_AXIS: return "eigenvalue on the imaginary axis";
    case SGN_ERR_UNSUPPORTED: return "unsupported option";
    }
    return "unknown status";
}

extern "C" const char *sgn_last_error(void) { return g_last_error.c_str(); }

extern "C" sgn_status sgn_init(sgn_handle *h, int device)
{
    return guard([&] {
        SGN_REQUIRE(h != nullptr, "sgn_init: null handle pointer");
        int n = 0;
        SGN_HIP(hipGetDeviceCount(&n));
        SGN_REQUIRE(device >= 0 && device < n, "sgn_init: no such device");
        SGN_HIP(hipSetDevice(device));
        auto *c = new Context();
        c->device = device;
        hipDeviceProp_t prop;
        SGN_HIP(hipGetDeviceProperties(&prop, device));
        c->num_cu = prop.multiProcessorCount;
        try {
            c->noalloc = noalloc_scratch(device);
        } catch (...) {
            delete c;
            throw;
        }
        *h = reinterpret_cast<sgn_handle>(c);
    });
}

extern "C" sgn_status sgn_finalize(sgn_handle h)
{
    return guard([&] {
        if (!h) return;
        auto *c = reinterpret_cast<Context *>(h);
        SGN_HIP(hipSetDevice(c->device));
        if (c->partials) SGN_HIP(hipFree(c->partials));
        if (c->scalars) SGN_HIP(hipFree(c->scalars));
        if (c->arena) SGN_HIP(hipFree(c->arena));
        if (c->small) SGN_HIP(hipFree(c->small));
        if (c->byte_counter) SGN_HIP(hipFree(c->byte_counter));
        for (auto &kv : c->basis_pools)
            for (void *b : kv.second) SGN_HIP(hipFree(b));
        if (c->capture_stream) SGN_HIP(hipStreamDestroy(c->capture_stream));
        for (auto &r : c->prof_recs) {
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
        for (auto e : c->event_pool) (void)hipEventDestroy(e);
        delete c;
    });
}

extern "C" sgn_status sgn_lattice_create(sgn_handle h, const sgn_lattice_desc *d, const void *links,
                                         unsigned prec_mask, void *stream, sgn_lattice *out)
{
    Lattice *lat = nullptr;
    sgn_status st = guard([&] {
        SGN_REQUIRE(h && d && links && out, "sgn_lattice_create: null argument");
        auto *ctx = reinterpret_cast<Context *>(h);
        int64_t V = 1;
        for (int i = 0; i < 4; ++i) {
            SGN_REQUIRE(d->dims[i] >= 2, "sgn_lattice_create: every extent must be >= 2");
            SGN_REQUIRE(d->bc[i] == 1 || d->bc[i] == -1, "sgn_lattice_create: bc must be +1 or -1");
            V *= d->dims[i];
        }
        SGN_REQUIRE(V <= (int64_t)(1 << 26), "sgn_lattice_create: volume above 2^26 sites");
        SGN_REQUIRE(std::isfinite(d->kappa), "sgn_lattice_create: kappa not finite");
        SGN_HIP(hipSetDevice(ctx->device));
        lat = new Lattice();
        lat->ctx = ctx;
        for (int i = 0; i < 4; ++i) {
            lat->L[i] = d->dims[i];
            lat->bc[i] = d->bc[i];
        }
        lat->kappa = d->kappa;
        lat->V = V;
        lat->S = component_stride(V);
        const int64_t S = lat->S;
        const unsigned pmask = prec_mask & 7u;
        const unsigned mask = pmask ? pmask : 7u;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int nthr = (int)(4 * V);
        dim3 g((nthr + 255) / 256), b(256);
        // two-row storage when every link is SU(3) to 1e-12
        lat->link_ne = 9;
        const bool temporal = (prec_mask & SGN_LINKS_TEMPORAL_GAUGE) != 0;
        bool su3 = false;
        if (!(prec_mask & SGN_LINKS_FULL) || temporal) {
            std::vector<double> bm(g.x);
            double *dbm = nullptr;
            if (hipMalloc(&dbm, sizeof(double) * g.x) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "su3 check"};
            hipLaunchKernelGGL(su3_check_kernel, g, b, 0, s, (const double2 *)links, nthr, dbm);
            const hipError_t e1 = hipGetLastError();
            const hipError_t e2 = hipMemcpyAsync(bm.data(), dbm, sizeof(double) * g.x, hipMemcpyDeviceToHost, s);
            const hipError_t e3 = hipStreamSynchronize(s);
            (void)hipFree(dbm);
            SGN_HIP(e1);
            SGN_HIP(e2);
            SGN_HIP(e3);
            double dev = 0.0;
            for (double v : bm) dev = std::max(dev, v);
            su3 = dev <= 1e-12;
            if (su3 && !(prec_mask & SGN_LINKS_FULL)) lat->link_ne = 6;
        }
        SGN_REQUIRE(su3 || !temporal, "sgn_lattice_create: the temporal gauge needs SU(3) links (to 1e-12)");
        void *fixed = nullptr;  // the links in the temporal gauge, canonical layout (freed on return)
        struct FreeOnExit {
            void *&p;
            ~FreeOnExit() { if (p) (void)hipFree(p); }
        } free_fixed{fixed};
        if (temporal) {
            const int vs = lat->L[0] * lat->L[1] * lat->L[2];
            if (hipMalloc(&lat->gauge, (size_t)V * 9 * 16) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "gauge rotation"};
            if (hipMalloc(&fixed, (size_t)V * 36 * 16) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "gauge-fixed links"};
            hipLaunchKernelGGL(tg_gauge_kernel, dim3((vs + 63) / 64), dim3(64), 0, s, (const double2 *)links,
                               (double2 *)lat->gauge, vs, lat->L[3]);
            hipLaunchKernelGGL(tg_links_kernel, g, b, 0, s, (const double2 *)links, (const double2 *)lat->gauge,
                               static_cast<double2 *>(fixed), (int)V, lat->L[0], lat->L[1], lat->L[2], lat->L[3]);
            SGN_HIP(hipGetLastError());
            links = fixed;
        }
        const size_t nel = (size_t)S * 4 * lat->link_ne;
        const int ne = lat->link_ne;
        if (mask & (1u << SGN_PREC_F64)) {
            if (hipMalloc(&lat->links64, nel * 16) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "links64"};
            SGN_HIP(hipMemsetAsync(lat->links64, 0, nel * 16, s));
            hipLaunchKernelGGL(pack_links_kernel<double2>, g, b, 0, s, (const double2 *)links,
                               (double2 *)lat->links64, (int)V, (int)S, ne);
        }
        if (mask & (1u << SGN_PREC_F32)) {
            if (hipMalloc(&lat->links32, nel * 8) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "links32"};
            SGN_HIP(hipMemsetAsync(lat->links32, 0, nel * 8, s));
            hipLaunchKernelGGL(pack_links_kernel<float2>, g, b, 0, s, (const double2 *)links,
                               (float2 *)lat->links32, (int)V, (int)S, ne);
        }
        if (mask & (1u << SGN_PREC_F32_H16)) {
            if (hipMalloc(&lat->links16, nel * 4) != hipSuccess) throw Failure{SGN_ERR_NOMEM, "links16"};
            SGN_HIP(hipMemsetAsync(lat->links16, 0, nel * 4, s));
            hipLaunchKernelGGL(pack_links_kernel<__half2>, g, b, 0, s, (const double2 *)links,
                               (__half2 *)lat->links16, (int)V, (int)S, ne);
        }
        SGN_HIP(hipGetLastError());
        SGN_HIP(hipStreamSynchronize(s));
        *out = reinterpret_cast<sgn_lattice>(lat);
    });
    if (st != SGN_OK && lat) sgn_lattice_destroy(reinterpret_cast<sgn_lattice>(lat));
    return st;
}

extern "C" sgn_status sgn_lattice_destroy(sgn_lattice l)
{
    return guard([&] {
        if (!l) return;
        Lattice *lat = as_lattice(l);
        SGN_HIP(hipSetDevice(lat->ctx->device));
        for (void *p : {lat->links64, lat->links32, lat->links16, lat->gauge, lat->stage_in, lat->stage_out})
            if (p) SGN_HIP(hipFree(p));
        delete lat;
    });
}

extern "C" int64_t sgn_lattice_volume(sgn_lattice l) { return l ? as_lattice(l)->V : 0; }

extern "C" int sgn_lattice_link_elements(sgn_lattice l) { return l ? as_lattice(l)->link_ne : 0; }

extern "C" size_t sgn_spinor_bytes(sgn_lattice l, sgn_prec p) { return l ? spinor_bytes(as_lattice(l)->S, p) : 0; }

extern "C" sgn_status sgn_spinor_pack(sgn_lattice l, const void *canon, void *internal, sgn_prec p, void *stream)
{
    return guard([&] {
        SGN_REQUIRE(l && canon && internal, "sgn_spinor_pack: null argument");
        Lattice &lat = *as_lattice(l);
        SGN_HIP(hipSetDevice(lat.ctx->device));
        pack_spinor(lat, canon, internal, p, static_cast<hipStream_t>(stream));
    });
}

extern "C" sgn_status sgn_spinor_unpack(sgn_lattice l, const void *internal, void *canon, sgn_prec p, void *stream)
{
    return guard([&] {
        SGN_REQUIRE(l && canon && internal, "sgn_spinor_unpack: null argument");
        Lattice &lat = *as_lattice(l);
        SGN_HIP(hipSetDevice(lat.ctx->device));
        unpack_spinor(lat, internal, canon, p, static_cast<hipStream_t>(stream));
    });
}

// ----------------------------------------------------------------------------- profiling
namespace sgn {

int Context::prof_start(hipStream_t s, int cls, bool stamped)
{
    if (!prof) return -1;
    if (prof_calls[cls]++ % prof_every != 0) return -1;
    ProfRec r{};
    for (hipEvent_t *e : {&r.start, &r.stop}) {
        if (!event_pool.empty()) {
            *e = event_pool.back();
            event_pool.pop_back();
        } else {
            SGN_HIP(hipEventCreate(e));
        }
    }
    r.stamped = stamped;
    if (!stamped) SGN_HIP(hipEventRecord(r.start, s));
    prof_recs.push_back(r);
    return (int)prof_recs.size() - 1;
}

LaunchStamp Context::prof_stamp(int rec) const
{
    LaunchStamp ev;
    if (rec >= 0 && prof_recs[rec].stamped) {
        ev.start = prof_recs[rec].start;
        ev.stop = prof_recs[rec].stop;
    }
    return ev;
}

void Context::prof_stop(int rec, hipStream_t s, int cls, double bytes, double flops, bool device_bytes,
                        double bytes_stored)
{
    if (rec < 0) return;
    ProfRec &r = prof_recs[rec];
    r.cls = cls;
    r.bytes = bytes;
    r.bytes_stored = bytes_stored < 0.0 ? bytes : bytes_stored;
    r.flops = flops;
    r.device_bytes = device_bytes;
    if (!r.stamped) SGN_HIP(hipEventRecord(r.stop, s));
}

void Context::prof_collect()
{
    for (ProfRec &r : prof_recs) {
        SGN_HIP(hipEventSynchronize(r.stop));
        float ms = 0.f;
        SGN_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
        acc_ms[r.cls] += ms;
        acc_bytes[r.cls] += r.bytes;
        acc_bytes_stored[r.cls] += r.bytes_stored;
        acc_flops[r.cls] += r.flops;
        acc_launches[r.cls] += 1;
        event_pool.push_back(r.start);
        event_pool.push_back(r.stop);
    }
    prof_recs.clear();
    if (byte_counter) {
        unsigned long long b = 0;
        SGN_HIP(hipMemcpy(&b, byte_counter, sizeof(b), hipMemcpyDeviceToHost));
        acc_bytes[SGN_K_SHIFT_UPDATE] += (double)b;
        acc_bytes_stored[SGN_K_SHIFT_UPDATE] += (double)b;
        const unsigned long long z = 0;
        SGN_HIP(hipMemcpy(byte_counter, &z, sizeof(z), hipMemcpyHostToDevice));
    }
}

}  // namespace sgn

extern "C" sgn_status sgn_profile_enable(sgn_handle h, int enable)
{
    return guard([&] {
        SGN_REQUIRE(h != nullptr, "sgn_profile_enable: null handle");
        auto *c = reinterpret_cast<Context *>(h);
        SGN_HIP(hipSetDevice(c->device));
        SGN_HIP(hipDeviceSynchronize());
        c->prof_collect();
        for (int k = 0; k < SGN_K_COUNT; ++k) {
            c->acc_ms[k] = c->acc_bytes[k] = c->acc_flops[k] = c->acc_bytes_stored[k] = 0.0;
            c->acc_launches[k] = 0;
        }
        if (enable && !c->byte_counter) {
            if (hipMalloc(&c->byte_counter, sizeof(unsigned long long)) != hipSuccess)
                throw Failure{SGN_ERR_NOMEM, "profiling counter"};
            const unsigned long long z = 0;
            SGN_HIP(hipMemcpy(c->byte_counter, &z, sizeof(z), hipMemcpyHostToDevice));
        }
        c->prof = enable != 0;
        c->prof_every = enable > 1 ? enable : 1;
        for (int k = 0; k < SGN_K_COUNT; ++k) c->prof_calls[k] = 0;
    });
}

extern "C" sgn_status sgn_profile_read(sgn_handle h, sgn_kernel_profile *out)
{
    return guard([&] {
        SGN_REQUIRE(h != nullptr && out != nullptr, "sgn_profile_read: null argument");
        auto *c = reinterpret_cast<Context *>(h);
        SGN_HIP(hipSetDevice(c->device));
        c->prof_collect();
        for (int k = 0; k < SGN_K_COUNT; ++k) {
            out[k].launches = c->acc_launches[k];
            out[k].total_ms = c->acc_ms[k];
            out[k].bytes = c->acc_bytes[k];
            out[k].flops = c->acc_flops[k];
            out[k].calls = c->prof_calls[k];
            out[k].bytes_stored = c->acc_bytes_stored[k];
        }
    });
}
