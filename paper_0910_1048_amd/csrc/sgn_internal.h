// Internal declarations of libsgn (gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sgn.h"

namespace sgn {

// ----------------------------------------------------------------------------- errors
void set_error(const std::string &msg);

struct Failure {
    sgn_status st;
    std::string msg;
};

#define SGN_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::sgn::Failure{SGN_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define SGN_REQUIRE(cond, msg)                                                              \
    do {                                                                                    \
        if (!(cond)) throw ::sgn::Failure{SGN_ERR_INVALID, (msg)};                          \
    } while (0)

// Run `body`, translating Failure / std::exception into a status code.
template <typename F>
sgn_status guard(F &&body)
{
    try {
        body();
        return SGN_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return SGN_ERR_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return SGN_ERR_INVALID;
    }
}

// ----------------------------------------------------------------------------- complex
template <typename R>
struct cpx {
    R r, i;
};

template <typename R> __host__ __device__ inline cpx<R> mk(R r, R i) { return cpx<R>{r, i}; }
template <typename R> __host__ __device__ inline cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.r + b.r, a.i + b.i}; }
template <typename R> __host__ __device__ inline cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.r - b.r, a.i - b.i}; }
template <typename R> __host__ __device__ inline cpx<R> operator-(cpx<R> a) { return {-a.r, -a.i}; }
template <typename R> __host__ __device__ inline cpx<R> operator*(cpx<R> a, cpx<R> b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename R> __host__ __device__ inline cpx<R> operator*(R s, cpx<R> a) { return {s * a.r, s * a.i}; }
template <typename R> __host__ __device__ inline cpx<R> conj(cpx<R> a) { return {a.r, -a.i}; }
// conj(a) * b
template <typename R> __host__ __device__ inline cpx<R> cmulc(cpx<R> a, cpx<R> b)
{
    return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
template <typename R> __host__ __device__ inline cpx<R> times_i(cpx<R> a) { return {-a.i, a.r}; }
template <typename R> __host__ __device__ inline cpx<R> times_mi(cpx<R> a) { return {a.i, -a.r}; }
template <typename R> __host__ __device__ inline R norm2(cpx<R> a) { return a.r * a.r + a.i * a.i; }
template <typename A, typename B> __host__ __device__ inline cpx<A> cast(cpx<B> b)
{
    return {static_cast<A>(b.r), static_cast<A>(b.i)};
}

using z64 = cpx<double>;

// ----------------------------------------------------------------------------- objects
struct ProfRec {
    int cls;
    hipEvent_t start, stop;
    double bytes, flops, bytes_stored;
    bool device_bytes;  // bytes accumulated by the kernel itself into byte_counter
    bool stamped;       // the events are stamped by the dispatch of one kernel (launch_k)
};

// Events that the dispatch of one kernel stamps with the kernel's own start and end.
struct LaunchStamp {
    hipEvent_t start = nullptr, stop = nullptr;
};

struct Context {
    int device = 0;
    int num_cu = 0;
    // profiling of the library's own launches (sgn_profile_enable)
    bool prof = false;
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> event_pool;
    unsigned long long *byte_counter = nullptr;  // device, bytes reported by kernels
    double acc_ms[SGN_K_COUNT] = {};
    double acc_bytes[SGN_K_COUNT] = {};
    double acc_bytes_stored[SGN_K_COUNT] = {};
    double acc_flops[SGN_K_COUNT] = {};
    long long acc_launches[SGN_K_COUNT] = {};
    // returns -1 when profiling is off or this launch of class cls is not sampled
    int prof_every = 1;
    long long prof_calls[SGN_K_COUNT] = {};
    // stamped: the caller launches exactly one kernel with prof_stamp(rec) (launch_k); otherwise
    // event markers are recorded on s around whatever the caller launches
    int prof_start(hipStream_t s, int cls, bool stamped = false);
    LaunchStamp prof_stamp(int rec) const;
    // bytes: algorithmic bytes (links as nine entries); bytes_stored: in the stored format (< 0: = bytes)
    void prof_stop(int rec, hipStream_t s, int cls, double bytes, double flops, bool device_bytes = false,
                   double bytes_stored = -1.0);
    void prof_collect();
    // scratch device buffers owned by the context, grown on demand
    void *partials = nullptr;
    size_t partials_bytes = 0;
    void *scalars = nullptr;  // device scalars of the solvers
    size_t scalars_bytes = 0;
    void *ensure_partials(size_t bytes);
    void *ensure_scalars(size_t bytes);
    // solver workspace arena, grown on demand and kept between calls
    void *arena = nullptr;
    size_t arena_bytes = 0;
    void *ensure_arena(size_t bytes);
    // small device scratch of the deflation prologue (coefficients, probes), grown on demand
    void *small = nullptr;
    size_t small_bytes = 0;
    void *ensure_small(size_t bytes);
    // stored Krylov vectors of the multishift solver, one pool per vector size,
    // kept between calls
    std::map<size_t, std::vector<void *>> basis_pools;
    // stream on which solver iterations are captured into HIP graphs
    hipStream_t capture_stream = nullptr;
    // this device's address of the static staging array of wilson_apply_noalloc
    void *noalloc = nullptr;
    // stencil launch shapes chosen by sgn_autotune, per {Lx, Ly, Lz, Lt, precision, multi-RHS}:
    // the block's site cap (0: the default plan) and, for the multi-RHS form with FP16 links,
    // whether the links are held in registers (-1: default)
    struct TunedShape {
        int max_sites = 0;
        int regs = -1;
        int tslices = 1;  // staged blocks of 1 t-slice, or bricks of 2
        int unstaged = 0;  // 1: the kernel without LDS staging (every neighbour through the caches)
    };
    std::map<std::vector<int>, TunedShape> tuned;
    TunedShape tuned_shape(const int L[4], sgn_prec p, bool multi) const
    {
        auto it = tuned.find({L[0], L[1], L[2], L[3], (int)p, multi ? 1 : 0});
        return it == tuned.end() ? TunedShape{} : it->second;
    }
};

struct Lattice {
    Context *ctx = nullptr;
    int L[4] = {0, 0, 0, 0};
    int bc[4] = {1, 1, 1, -1};
    double kappa = 0.0;
    int64_t V = 0;
    // component stride of every internal field array, >= V (padded so that the
    // 12 spinor and 36 link component arrays of one site do not fall into the
    // same L2 set)
    int64_t S = 0;
    int link_ne = 9;          // complex entries stored per link: 6 (rows 0, 1 of an SU(3) matrix) or 9
    void *links64 = nullptr;  // [4][link_ne][S] double2
    void *links32 = nullptr;  // [4][link_ne][S] float2
    void *links16 = nullptr;  // [4][link_ne][S] __half2
    // temporal gauge (SGN_LINKS_TEMPORAL_GAUGE): the colour rotation G(x), [V][3][3] double2, that the
    // stored links and every internal field are expressed in; null otherwise
    void *gauge = nullptr;
    // canonical <-> internal staging for wilson_apply in canonical layout
    void *stage_in = nullptr, *stage_out = nullptr;
    size_t stage_bytes = 0;
    void ensure_stage(size_t bytes);
    // parameters of multi-RHS launches on this lattice (wilson_apply_multi)
    mutable std::shared_ptr<class StencilBatch> multi;
};

inline size_t spinor_bytes(int64_t S, sgn_prec p) { return (size_t)S * 12 * (p == SGN_PREC_F64 ? 16 : 8); }

// component stride for a lattice of V sites (a multiple of 64 sites, offset by an odd
// multiple of 64 sites from a multiple of 128 sites for volumes where aliasing matters)
inline int64_t component_stride(int64_t V)
{
    if (V < 4096) return V;
    const int64_t r = (V + 63) / 64 * 64;
    return r + ((r / 64) % 2 == 0 ? 320 : 256);
}

// ----------------------------------------------------------------------------- launches
// Operator selection for one stencil application.
struct OpSpec {
    double mu = 0.0;     // chemical potential actually used (the adjoint passes -mu)
    bool g5_out = true;  // multiply the result by gamma5
    bool g5_in = false;  // multiply the input by gamma5 first
};

// Epilogue of a stencil application:  out = a * Op(in) + b * z   (z optional),
// optionally accumulating per-block partial sums of  conj(w) . out  (FP64).
struct Epilogue {
    double a = 1.0;
    z64 b = {0.0, 0.0};
    const z64 *b_dev = nullptr;   // if set, b is read from device memory (times b)
    const void *z = nullptr;      // same precision/layout as out
    const void *w = nullptr;      // dot partner, same precision/layout as out
    z64 *partials = nullptr;      // one z64 per block when w != nullptr (two with norm)
    const z64 *in_scale = nullptr;  // if set: Op(in) is multiplied by *in_scale (device)
    bool norm = false;            // with w: also ||out||^2, partials[2b] = dot, partials[2b+1] = {norm, 0}
};

// Launch the stencil on internal-layout fields.  Returns the number of blocks
// (= number of partials written when ep.w is set).
// nr (1..16) right-hand sides in one launch sharing every link load; each has
// its own operator (mu, gamma5 flags), input, output and epilogue.
int dslash_launch_multi(const Lattice &lat, sgn_prec p, int nr, const OpSpec *op, const void *const *in,
                        void *const *out, const Epilogue *ep, hipStream_t s);
int dslash_launch(const Lattice &lat, sgn_prec p, const OpSpec &op, const void *in, void *out,
                  const Epilogue &ep, hipStream_t s);
int dslash_blocks(const Lattice &lat);

// One single-RHS stencil application of a batch.
struct StencilJob {
    const Lattice *lat = nullptr;
    OpSpec op;
    const void *in = nullptr;
    void *out = nullptr;
    Epilogue ep;
};

// Independent applications of one precision (own lattices, fields, epilogues)
// launched together: one launch, with the applications on one lattice grouped
// into multi-RHS groups of up to 16 (one block walks all right-hand sides of its
// group, sharing the link loads) and blockIdx.y selecting the group; the
// parameters stay in device memory between launches.  Falls back to one launch
// per application when some lattice has no staged block shape.
class StencilBatch {
  public:
    StencilBatch() = default;
    ~StencilBatch();
    StencilBatch(const StencilBatch &) = delete;
    StencilBatch &operator=(const StencilBatch &) = delete;
    void prepare(const std::vector<StencilJob> &jobs, sgn_prec p);  // synchronous upload
    void launch(hipStream_t s) const;
    int blocks(size_t k) const { return nblk_[k]; }  // partials written by application k
    size_t size() const { return jobs_.size(); }

  private:
    std::vector<StencilJob> jobs_;
    std::vector<int> nblk_;
    sgn_prec prec_ = SGN_PREC_F64;
    void *dev_ = nullptr;
    size_t dev_bytes_ = 0;
    std::vector<char> uploaded_;  // the parameters now on the device
    int gx_ = 0, threads_ = 0, ngroups_ = 0;
    size_t lds_ = 0;
    bool batched_ = false, epi_ = false, dot_ = false, regs_ = false;
    double bytes_ = 0.0, flops_ = 0.0, bytes_stored_ = 0.0;
};

// Single shifted system (c^2 H^2 - sigma) x = y of the rational methods, FP64, internal layout
// (12 S entries).  shift_residual64: out = y - (c^2 H^2 - sigma) x, returns ||out|| (tmp: one
// intermediate field; synchronises).  refine_shift64: x += e with (c^2 H^2 - sigma) e = r by FP64
// BiCGStab until ||r|| <= target or maxiter; r holds the true residual of x on entry and is
// overwritten; work holds six fields; returns the iterations and adds the applications of H to
// *matvecs.
double shift_residual64(Lattice &lat, const OpSpec &op, double c2, double sigma, const void *y, const void *x,
                        void *out, void *tmp, hipStream_t s);
int refine_shift64(Lattice &lat, const OpSpec &op, double c2, double sigma, void *r, void *x, double target,
                   int maxiter, void *work, void *tmp, hipStream_t s, int *matvecs);

void pack_spinor(const Lattice &lat, const void *canon, void *internal, sgn_prec p, hipStream_t s);
// device address of wilson_apply_noalloc's static staging array on `device` (must be current);
// taken once per device
void *noalloc_scratch(int device);
void unpack_spinor(const Lattice &lat, const void *internal, void *canon, sgn_prec p, hipStream_t s);

inline Lattice *as_lattice(sgn_lattice l) { return reinterpret_cast<Lattice *>(l); }

// Run launch(stream) from a HIP graph: captured once on the context's capture stream into exec
// (which the caller keeps, and destroys when its launches change), then launched on s.  Without
// use_graph, or with launch profiling on (its events are not captured), launch runs on s directly.
template <typename F>
void replay_or_capture(Context &ctx, hipGraphExec_t &exec, bool use_graph, hipStream_t s, F &&launch)
{
    if (!use_graph || ctx.prof) {
        launch(s);
        return;
    }
    if (!exec) {
        if (!ctx.capture_stream) SGN_HIP(hipStreamCreate(&ctx.capture_stream));
        hipStream_t cs = ctx.capture_stream;
        hipGraph_t g = nullptr;
        SGN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            launch(cs);
        } catch (...) {
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        SGN_HIP(hipStreamEndCapture(cs, &g));
        const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        SGN_HIP(e);
    }
    SGN_HIP(hipGraphLaunch(exec, s));
}

}  // namespace sgn
