/*
 * sgn.h -- C ABI of libsgn: sign(H_W) b for the Wilson kernel H_W = gamma5 D_W(mu)
 * at nonzero chemical potential, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Bloch, Breu, Frommer, Heybrock, Schaefer, Wettig, "Short-recurrence
 * Krylov subspace methods for the overlap Dirac operator at nonzero chemical
 * potential".  Section and equation names below refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers marked (device) are HIP device pointers; (host) are host memory.
 *    The caller owns every buffer it passes; the library owns the handle, the
 *    lattice objects and all internal workspaces.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are stream-ordered and asynchronous unless stated otherwise.
 *  - Complex numbers are interleaved (re, im) doubles (complex128) or floats
 *    (complex64).
 *  - Canonical field layout (the boundary layout):
 *      spinor  [t][z][y][x][spin 4][colour 3]          complex
 *      links   [t][z][y][x][nu 4][3][3] row-major U_nu(x), nu = x, y, z, t
 *    flat site index x + Lx*(y + Ly*(z + Lz*t)); n = 12 * V complex entries.
 *  - Every call returns an sgn_status; nothing throws across the ABI.  On an
 *    error the output buffers are unspecified unless stated otherwise, and
 *    sgn_last_error() returns a message for the calling thread.
 *
 * The operator (the paper takes it from its reference on the overlap operator
 * at nonzero mu and does not print it; this library implements):
 *   (D_W psi)(x) = psi(x) - kappa sum_nu [ w^f_nu (1-gamma_nu) U_nu(x) psi(x+nu)
 *                                        + w^b_nu (1+gamma_nu) U_nu(x-nu)^H psi(x-nu) ]
 *   w^f_t = e^{-mu}, w^b_t = e^{+mu}, spatial weights 1; hops that wrap around
 *   direction nu carry the factor bc[nu] (+1 periodic, -1 antiperiodic).
 *   Gamma matrices in the DeGrand-Rossi chiral basis, gamma5 = diag(1,1,-1,-1).
 *   H_W(mu)^H = H_W(-mu) (gamma5-hermiticity).
 */
#ifndef SGN_H
#define SGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGN_OK = 0,
    SGN_ERR_INVALID = 1,        /* bad argument, NaN input, inconsistent deflation set */
    SGN_ERR_HIP = 2,            /* a HIP runtime call failed */
    SGN_ERR_NOMEM = 3,          /* device allocation failed */
    SGN_ERR_BREAKDOWN = 4,      /* two-sided Lanczos / BiCG breakdown */
    SGN_ERR_NOT_CONVERGED = 5,  /* iteration limit reached; x holds the last iterate */
    SGN_ERR_IMAG_AXIS = 6,      /* sign undefined: eigenvalue on the imaginary axis */
    SGN_ERR_UNSUPPORTED = 7     /* option combination not implemented */
} sgn_status;

/* Arithmetic of the stencil and of the vectors it touches. */
typedef enum {
    SGN_PREC_F64 = 0,       /* complex128 spinors, complex128 links */
    SGN_PREC_F32 = 1,       /* complex64 spinors, complex64 links   */
    SGN_PREC_F32_H16 = 2    /* complex64 spinors, IEEE half links, FP32 accumulation */
} sgn_prec;

typedef struct sgn_context_s *sgn_handle;
typedef struct sgn_lattice_s *sgn_lattice;

typedef struct {
    int dims[4];      /* Lx, Ly, Lz, Lt (each >= 2) */
    int bc[4];        /* +1 or -1 per direction (default use: 1, 1, 1, -1) */
    double kappa;     /* hopping parameter, kappa = 1/(8 - 2 rho) */
} sgn_lattice_desc;

/* flags for wilson_apply / wilson_apply_dag */
#define SGN_NO_GAMMA5       1u  /* apply D_W(mu) instead of H_W = gamma5 D_W(mu) */
#define SGN_INTERNAL_LAYOUT 2u  /* in/out are in the library's field layout (sgn_spinor_pack) */

/* ------------------------------------------------------------------ context */
/* Create a context on HIP device `device`.  Owns the solver workspaces (device
 * buffers grown on demand and kept between calls).  Not thread-safe: use one
 * context per thread. */
sgn_status sgn_init(sgn_handle *h, int device);
sgn_status sgn_finalize(sgn_handle h);
const char *sgn_status_string(sgn_status s);
const char *sgn_last_error(void);

/* ------------------------------------------------------------------ lattice */
/* Pack the gauge field `links` (device, canonical layout, complex128) into the
 * library's internal copies.  `prec_mask` is a bit mask of (1 << sgn_prec)
 * values saying which link precisions to keep (0 = all), optionally or-ed with
 * SGN_LINKS_FULL.  When every link is in SU(3) to 1e-12 (U U^H = I, det U = 1)
 * only its first two rows are stored and the third is rebuilt in the stencil as
 * the complex conjugate of their cross product (unitarity and unit determinant
 * fix it); otherwise, or with SGN_LINKS_FULL, all nine entries are stored.  The
 * caller may free `links` once the call returns (the call synchronises `stream`). */
#define SGN_LINKS_FULL 0x100u
/* SGN_LINKS_TEMPORAL_GAUGE (or-ed into prec_mask; SU(3) links only, else SGN_ERR_INVALID): the
 * lattice stores the field after the colour rotation G(x) in SU(3) with G(x, t=0) = 1 and
 * G(x, t+1) = G(x, t) U_t(x, t), so that every time link off the last time slice is the unit matrix
 * and the stencil skips its load and product.  The operator becomes G H_W G^H and sign(H_W) b =
 * G^H sign(G H_W G^H) G b; sgn_spinor_pack applies G and sgn_spinor_unpack G^H (in FP64), so every
 * result in the canonical layout is that of the field as given, up to rounding, and internal-layout
 * fields hold rotated spinors.  Costs one [V][3][3] complex128 array for G. */
#define SGN_LINKS_TEMPORAL_GAUGE 0x200u
sgn_status sgn_lattice_create(sgn_handle h, const sgn_lattice_desc *d, const void *links,
                              unsigned prec_mask, void *stream, sgn_lattice *out);
sgn_status sgn_lattice_destroy(sgn_lattice lat);
/* sites V and bytes of one spinor in the internal layout for precision p */
int64_t sgn_lattice_volume(sgn_lattice lat);
/* complex entries stored per link: 6 (two rows, SU(3) links) or 9 */
int sgn_lattice_link_elements(sgn_lattice lat);
size_t sgn_spinor_bytes(sgn_lattice lat, sgn_prec p);

/* Canonical <-> internal layout.  `canon` is complex128 for SGN_PREC_F64 and
 * complex64 otherwise; `internal` holds sgn_spinor_bytes(lat, p) bytes.  On a
 * temporal-gauge lattice (SGN_LINKS_TEMPORAL_GAUGE) pack stores G(x) psi(x) and unpack
 * returns G(x)^H of what it reads, each site's colour rotation done in FP64 (a round
 * trip is then exact only up to rounding). */
sgn_status sgn_spinor_pack(sgn_lattice lat, const void *canon, void *internal, sgn_prec p, void *stream);
sgn_status sgn_spinor_unpack(sgn_lattice lat, const void *internal, void *canon, sgn_prec p, void *stream);

/* ------------------------------------------------------------------ operator */
/* out = H_W(mu) in (flags: SGN_NO_GAMMA5 -> D_W(mu) in).  in/out (device) are
 * canonical complex128 for SGN_PREC_F64 and complex64 otherwise, or internal
 * layout with SGN_INTERNAL_LAYOUT.  in and out must not overlap. */
sgn_status wilson_apply(sgn_lattice lat, double mu, const void *in, void *out, sgn_prec p,
                        unsigned flags, void *stream);
/* out = H_W(mu)^H in = H_W(-mu) in  (with SGN_NO_GAMMA5: D_W(mu)^H in). */
sgn_status wilson_apply_dag(sgn_lattice lat, double mu, const void *in, void *out, sgn_prec p,
                            unsigned flags, void *stream);

/* wilson_apply without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops or harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as wilson_apply; the
 * canonical <-> internal staging of in and out uses one static device array of
 * SGN_NOALLOC_MAX_BYTES bytes per GPU (held by every GPU the library runs on
 * until the process ends) instead of per-lattice buffers, so a canonical-layout
 * call needs 2 * sgn_spinor_bytes(lat, p) <= SGN_NOALLOC_MAX_BYTES (FP64: up to
 * 65536 sites, e.g. 16^4; FP32: about twice that), else SGN_ERR_INVALID.  With
 * SGN_INTERNAL_LAYOUT no staging is used and any lattice size is accepted.
 * All calls on one GPU share that array and each leaves its fields there:
 * calls that overlap in time on one GPU (unordered streams, several host
 * threads) race and must be serialised by the caller. */
#define SGN_NOALLOC_MAX_BYTES 25288704u
sgn_status wilson_apply_noalloc(sgn_lattice lat, double mu, const void *in, void *out, sgn_prec p,
                                unsigned flags, void *stream);

/* out[i] = H_W(mu[i]) in[i] for i < nrhs on one gauge field (flags: SGN_NO_GAMMA5
 * as above; SGN_INTERNAL_LAYOUT is required).  Right-hand sides are processed in
 * groups of up to 16 (multi-RHS stencil): a block of sites applies the operator to
 * every right-hand side of its group in turn, staging each one's spinors in LDS,
 * and loads the sites' links once for the group (with FP16 links they are held
 * in registers in their two-row form; set SGN_MULTI_LINK_REGS=0 in the
 * environment to read them again for each right-hand side), so a group moves
 * (2 S N + L) bytes per site for N spinors of S bytes and links of L bytes
 * instead of N (2 S + L).  Each right-hand side's result is bitwise that of its
 * own wilson_apply.  mu (host) holds nrhs values; in/out (host arrays of device
 * pointers) must not alias each other.  The group's parameters live in device
 * memory owned by the lattice; a call with other fields or mu than the previous
 * one waits for the device to finish the earlier launches before replacing them. */
sgn_status wilson_apply_multi(sgn_lattice lat, int nrhs, const double *mu, const void *const *in,
                              void *const *out, sgn_prec p, unsigned flags, void *stream);

/* ------------------------------------------------------------------ launch-shape tuning */
/* One candidate launch shape of the stencil and its measured time. */
typedef struct {
    int block_sites;          /* lattice sites per block, all its t-slices (0: the unstaged kernel) */
    int links_in_registers;   /* multi-RHS form: links held in registers (1) or read per right-hand side (0) */
    double us;                /* one application (all nrhs right-hand sides), microseconds */
    int chosen;               /* 1 for the fastest candidate, now used by the context */
    int t_slices;             /* 1: the block's sites lie in one t-slice; 2: a brick of the same sites at
                                 t and t + 1, whose time hops between the two slices read LDS */
} sgn_tune_candidate;

/* Autotune the stencil's launch shape for lattices of lat's dimensions, precision p
 * and nrhs right-hand sides per launch (1: the single form, 2..16: the multi-RHS
 * form, whose choice serves every group size): every candidate -- the distinct
 * block sizes (whole x-rows or x-y planes within the LDS budget, under site caps
 * of 576, 432, 384, 288, 192 and 96), each as one t-slice and, for even L_t, as a
 * brick of two, for nrhs = 1 also the kernel without LDS staging (block_sites 0),
 * and with FP16 two-row links and nrhs > 1 both link modes -- is
 * applied reps times (0: 20) to zero fields on `stream` and timed
 * with HIP events; the fastest is kept in the context and used by every later
 * launch of that shape class on lattices of these dimensions (the solvers, the
 * batched form, wilson_apply and wilson_apply_multi).  Until then a default shape
 * is used.  out (host, may be NULL if max_out = 0) receives up to max_out
 * candidates in the order tried, *n_out (may be NULL) their count.  Allocates
 * 2 * nrhs fields for the duration of the call and synchronises the device. */
sgn_status sgn_autotune(sgn_lattice lat, sgn_prec p, int nrhs, int reps, sgn_tune_candidate *out, int max_out,
                        int *n_out, void *stream);

/* Set the launch shape used for lattices of lat's dimensions in precision p (multi = 0: the
 * single-RHS form, 1: the multi-RHS form) by hand, as sgn_autotune would: blocks of at most
 * max_sites sites (0: no cap beyond the LDS budget and the launch bound; -1: the kernel without
 * LDS staging, one launch per right-hand side in the multi-RHS form), t_slices = 1 or 2
 * (bricks of two t-slices, even L_t), links_in_registers = -1 (default), 0 or 1 (multi-RHS form
 * with FP16 two-row links).  For replaying a saved tuning result or pinning a shape.
 * SGN_ERR_INVALID if no staged block of that shape fits the lattice.  Synchronises the device. */
sgn_status sgn_tune_set(sgn_lattice lat, sgn_prec p, int multi, int max_sites, int t_slices,
                        int links_in_registers);

/* ------------------------------------------------------------------ deflation and statistics */
/* LR deflation set (section "Deflation", oblique projector P = R L^H):
 * m right eigenvectors R and left eigenvectors L of H_W(mu) for its m
 * critical eigenvalues lambda, normalised so that L^H R = I_m.  L and R
 * (device) hold m canonical complex128 vectors back to back (vector i at
 * offset i*n); lambda (host) holds m complex128 values.  m = 0 or a NULL
 * pointer to the struct means no deflation.  The caller owns all arrays.
 * Used for x_P = R sign(Lambda) L^H b (Eq. exact_proj) and r = (I - P) b.
 * Every solver first checks the set: L^H R = I is probed with a fixed vector v
 * of unit-modulus entries, and an entry of L^H R v - v larger than
 * 1e-8 ||l_i|| ||R v|| is SGN_ERR_INVALID ("L^H R differs from the identity");
 * an eigenvalue with |Re lambda| <= 1e-12 max|lambda| is SGN_ERR_IMAG_AXIS.
 * The check costs about 3m + 3 vector passes and one stream synchronisation. */
typedef struct {
    int m;
    const void *L;
    const void *R;
    const double *lambda;
} sgn_deflation;

#define SGN_MAX_POLES 128

/* Per-call statistics (any pointer may be NULL). */
typedef struct {
    int iterations;          /* Krylov steps (Lanczos), Arnoldi steps (FOM), BiCG iterations */
    int matvecs;             /* applications of H_W or H_W^H */
    int restarts;            /* FOM restart cycles */
    int reliable_updates;    /* FP64 true-residual recomputations (mixed precision) */
    int refine_iterations;   /* multishift_solve with verify: iterations of the per-shift FP64 refinement */
    int nshift;
    double shift_residual[SGN_MAX_POLES]; /* final relative residual of each shifted system */
    double residual;         /* largest final relative residual (rational methods) */
    double min_abs_re;       /* smallest |Re| of the small matrix's eigenvalues (direct Lanczos) */
    double krylov_ms;        /* time in the Krylov iteration (host clock, includes device waits) */
    double small_ms;         /* time in the small dense sign / Hessenberg solves */
    double total_ms;
} sgn_stats;

/* ------------------------------------------------------------------ direct two-sided Lanczos */
typedef struct {
    int k;              /* maximal Krylov dimension, fixed a priori (>= 1) */
    sgn_prec prec;      /* SGN_PREC_F64: FP64 throughout.  SGN_PREC_F32 / _H16: the two stencils
                           per step run in FP32 (FP16 links), the recurrence stays FP64 */
    double tol;         /* > 0: stop early once the lift coefficients y = sign(T_j) e_1 change by
                           less than tol (relative) between checks */
    int check_every;    /* steps between such checks (used when tol > 0).  The next check_every
                           steps are queued before the host evaluates a check, so up to that many
                           steps beyond the stopping point run and are discarded (counted in
                           stats->matvecs, not in stats->iterations) */
    int two_pass;       /* nonzero: keep only three basis vectors; a second, identical pass of the
                           recurrence (the kernels are deterministic) rebuilds v_j and accumulates
                           x, at twice the stencil work (memory O(n) instead of O(k n)) */
} sgn_lanczos_opts;

/* Direct two-sided Lanczos-LR(m, k) (section "Direct application of the
 * two-sided Lanczos approach", recurrences (2sided1)-(2sided2)):
 *   x_P = R sign(Lambda) L^H b,  r = b - R L^H b,  shadow r~ = b - L R^H b,
 *   v_1 = r/||r||, w_1 = r~ scaled to v_1^H w_1 = 1, k steps of two-sided
 *   Lanczos with A = H_W(mu), A^H = H_W(-mu), T_k tridiagonal,
 *   x = x_P + ||r|| V_k sign(T_k) e_1.
 * b, x: device, canonical complex128.  The small sign is evaluated on the host
 * in FP64 (complex Schur form); the call synchronises `stream`.  The basis
 * vectors v_j (FP64) are taken from the context's pool as the steps proceed and
 * stay with the context after the call (memory follows the steps taken, at most
 * k vectors; SGN_ERR_NOMEM when one cannot be allocated).
 * Returns SGN_ERR_BREAKDOWN if |w^H v| < 1e-14 ||w|| ||v|| at some step,
 * SGN_ERR_IMAG_AXIS if a deflated eigenvalue or an eigenvalue of T_k has
 * |Re| <= 1e-12 of the norm. */
sgn_status sign_lanczos_2sided(sgn_lattice lat, double mu, const void *b, void *x, const sgn_deflation *defl,
                               const sgn_lanczos_opts *opts, sgn_stats *stats, void *stream);

/* sign(T) e_1 for a k x k complex tridiagonal T, on the host: the small-matrix
 * step of the direct two-sided Lanczos method (section "Short recurrences":
 * f(H_k) of the projected matrix), the routine sign_lanczos_2sided calls.
 * diag[k], sub[k-1] (T(i+1,i)) and sup[k-1] (T(i,i+1)) are interleaved
 * (re, im) doubles (sub, sup may be NULL when k = 1); y[k] receives the
 * result, by the complex Schur form of T (implicit single-shift QR, O(k^3)) and
 * the eigenvectors of its triangular factor.  *min_abs_re (may be NULL)
 * receives min |Re lambda|.  SGN_ERR_INVALID for k < 1, NULL arrays or entries that are not finite,
 * SGN_ERR_IMAG_AXIS if |Re lambda| <= 1e-12 ||T||_inf for an eigenvalue,
 * SGN_ERR_BREAKDOWN if the QR iteration does not converge. */
sgn_status sgn_small_sign(int k, const double *diag, const double *sub, const double *sup, double *y,
                          double *min_abs_re);

/* ------------------------------------------------------------------ rational approximation */
/* sign(t) ~ g_s(c t) = c t sum_i omega_i / (c^2 t^2 - sigma_i)   (Eqs. (neuberger_mit_c), (pfe_s)):
 * the shifted systems of the rational methods are (c^2 H_W^2 - sigma_i) x_i = c H_W r. */
typedef struct {
    int s;                          /* number of poles, 1 <= s <= SGN_MAX_POLES */
    double c;                       /* scale c > 0 */
    double alpha, beta;             /* spectral bounds the coefficients were built for (informational) */
    double omega[SGN_MAX_POLES];    /* weights omega_i > 0 */
    double sigma[SGN_MAX_POLES];    /* shifts sigma_i < 0 */
} sgn_rational;

/* Neuberger coefficients of Eq. (pfe_s) with the scale of the spectral-circle
 * heuristic: circle through alpha and beta (0 < alpha < beta), m = (alpha+beta)/2,
 * r = (beta-alpha)/2, c = ((m+r)(m-r))^{-1/2}  (section on the choice of the
 * rational function and the numerical-results section).  Host only. */
sgn_status sgn_rational_neuberger(int s, double alpha, double beta, sgn_rational *out);
/* Smallest s satisfying Eq. (no_of_poles) for accuracy eps on the circles
 * through alpha and beta (circle theorem).  Host only. */
sgn_status sgn_poles_needed(double alpha, double beta, double eps, int *s);
/* Neuberger coefficients as sgn_rational_neuberger with every omega_i multiplied by
 * 2/(2 - e_max), e_max = max |1 - g_s(ct)| over real t in [alpha, beta] (footnote on the
 * choice of c): the largest real-axis error drops from e_max to e_max/(2 - e_max).
 * *err (may be NULL) receives that error.  Host only. */
sgn_status sgn_rational_neuberger_rescaled(int s, double alpha, double beta, sgn_rational *out, double *err);
/* Zolotarev's best uniform rational approximation of sign on [-beta,-alpha] u
 * [alpha,beta] with s poles in t^2 (the alternative named in the numerical-results
 * section for spectra close to the real axis), in the same partial-fraction form:
 * c = 1/beta, sigma_i = -c_{2i-1} with c_l = k^2 sn^2(l K'/(2s); k') / cn^2(l K'/(2s); k'),
 * k = alpha/beta, k' = sqrt(1-k^2), K' = K(k'); omega_i = D times the residues of the
 * product form, D normalising the error to equioscillate.  *err (may be NULL)
 * receives the uniform error on the two intervals.  Host only. */
sgn_status sgn_rational_zolotarev(int s, double alpha, double beta, sgn_rational *out, double *err);

/* ------------------------------------------------------------------ critical eigenpairs */
typedef struct {
    int m;             /* eigenpairs wanted, m >= 1 */
    int nev;           /* Ritz pairs kept per restart, nev > m (0: m + max(20, m), at most kmax - 2) */
    int kmax;          /* Arnoldi basis size, nev + 2 <= kmax <= 1024 and below 12 V
                          (0: 2 (m + max(20, m)) + 16, held below both limits) */
    double tol;        /* Ritz residual of H_W^2 <= tol |theta| for the m + 2 wanted (0: 1e-10) */
    int max_restarts;  /* per side (0: 1000) */
    unsigned seed;     /* start vectors (a fixed pseudo-random sequence per seed) */
} sgn_eig_opts;

/* Left and right eigenvectors of H_W(mu) for its m critical eigenvalues, the m
 * closest to the imaginary axis (section "Deflation"), in the format of
 * sgn_deflation: L, R (device) receive m canonical complex128 vectors each,
 * back to back, with L^H R = I_m and unit right vectors; lambda (host) receives
 * m complex128 values ordered by |Re lambda|.  Method: implicitly restarted
 * Arnoldi with exact shifts on H_W(mu)^2 and on H_W(-mu)^2 = (H_W^H)^2 for the
 * eigenvalues of smallest real part of the square, Rayleigh-Ritz with H_W on each
 * invariant subspace, then the oblique projection that pairs the two.  *alpha
 * (may be NULL) receives the smallest modulus among the right Ritz values kept
 * but not selected, an estimate of the smallest non-deflated |lambda|.
 * stats: iterations = Arnoldi steps, restarts, matvecs, residual = largest
 * ||H r - lambda r|| / (|lambda| ||r||) over both sides.  The m-th and (m+1)-th
 * eigenvalues should be separated: a cut inside a cluster leaves the projector
 * ill-determined.  SGN_ERR_NOT_CONVERGED if a side did not converge within
 * max_restarts (outputs hold the last approximation), or if it has fewer than m
 * Ritz pairs with residual <= 1e-4 |theta| (outputs not written; stats hold the
 * work done and sgn_last_error the count), SGN_ERR_BREAKDOWN if the
 * two subspaces do not pair (singular L^H R).  Synchronises `stream`. */
sgn_status sgn_critical_eigenpairs(sgn_lattice lat, double mu, const sgn_eig_opts *o, void *L, void *R,
                                   double *lambda, double *alpha, sgn_stats *stats, void *stream);

/* ------------------------------------------------------------------ restarted FOM (Arnoldi) */
typedef struct {
    int kmax;           /* Arnoldi steps per restart cycle (k_max) */
    double tol;         /* every shifted residual |rho_i| ||r|| <= tol ||c H (I-P) b|| */
    int max_restarts;   /* cycles (0: 1000) */
    sgn_prec prec;      /* SGN_PREC_F64: FP64 throughout.  SGN_PREC_F32: cycles start in FP64; once every
                           shifted residual is below theta32 ||y|| the basis, the stencil and the
                           Gram-Schmidt vectors are FP32 (FP64 sums, FP64 Hessenberg and x).
                           SGN_PREC_F32_H16: as F32, with FP16 links below theta16 */
    double theta32;     /* default 1e-3 if <= 0 */
    double theta16;     /* default 1e-6 if <= 0 */
} sgn_arnoldi_opts;

/* Restarted FOM-LR(m, k) (section "Restarted Arnoldi with rational functions"):
 * x = x_P + sum_i omega_i x_i with (c^2 H_W^2 - sigma_i) x_i = c H_W (I-P) b, all
 * shifts from one restarted Arnoldi process (classical Gram-Schmidt with one
 * reorthogonalisation, its second-pass coefficients taken from the basis's Gram
 * matrix: two passes over the basis per step) on c^2 H_W^2; the collinear restart of Eq. (collinearity); the projection step
 * r = (I-P) v_{k+1} after every cycle.  b, x: device canonical complex128.
 * The shifted Hessenberg systems are solved on the host each cycle; the call
 * synchronises `stream`.  SGN_ERR_NOT_CONVERGED after max_restarts cycles
 * (x holds the last iterate).  stats->restarts counts the cycles and
 * stats->reliable_updates those run with the FP32 basis. */
sgn_status sign_arnoldi_rational(sgn_lattice lat, double mu, const void *b, void *x, const sgn_rational *r,
                                 const sgn_deflation *defl, const sgn_arnoldi_opts *o, sgn_stats *stats,
                                 void *stream);

/* Restarted GMRES-LR(m, k) (Algorithm "Restarted GMRES-LR", section "Restarted
 * Arnoldi with rational functions", after Frommer and Glassner): the same
 * restarted Arnoldi process on c^2 H_W^2 as sign_arnoldi_rational, but the seed
 * system (the shift of smallest modulus) takes the minimal-residual iterate of
 * each cycle, ||beta e_1 - (Hh_k - sigma Ih_k) y|| over y, and every other shift
 * solves the (k+1) x (k+1) system that keeps its residual collinear to the
 * seed's, r_i = rho_i r_seed.  Restart vector v_1 = (I-P) r / beta with r the
 * seed's residual V_{k+1} z and beta = ||r|| taken before the projection.
 * Converged when |rho_i| beta <= tol ||c H (I-P) b|| for every shift (rho = 1 for
 * the seed).  Arguments, layout, precision schedule, statistics and errors as for
 * sign_arnoldi_rational; SGN_ERR_BREAKDOWN if a small system is singular. */
sgn_status sign_gmres_rational(sgn_lattice lat, double mu, const void *b, void *x, const sgn_rational *r,
                               const sgn_deflation *defl, const sgn_arnoldi_opts *o, sgn_stats *stats,
                               void *stream);

/* ------------------------------------------------------------------ multishift BiCG */
typedef struct {
    sgn_lattice lat;
    double mu;
    const void *b;              /* device, canonical complex128 */
    void *x;                    /* device, canonical complex128: x_P + sum_i omega_i x_i */
    const sgn_deflation *defl;  /* may be NULL */
    void *const *x_shift;       /* NULL, or s device pointers receiving the x_i (canonical complex128) */
} sgn_problem;

typedef struct {
    double tol;         /* every shifted system: ||c H r - (c^2 H^2 - sigma_i) x_i|| <= tol ||c H r|| */
    int maxiter;        /* BiCG iterations */
    sgn_prec prec;      /* SGN_PREC_F64: FP64 throughout.  SGN_PREC_F32: FP64 while the seed residual is
                           above theta32, then FP32 vectors and stencil with FP64 reliable updates.
                           SGN_PREC_F32_H16: as F32, and FP16 links once below theta16 */
    double theta32;     /* relative seed residual at which FP32 takes over (default 1e-3 if <= 0) */
    double theta16;     /* relative seed residual at which FP16 links take over (default 1e-6 if <= 0) */
    double delta;       /* reliable update when the seed residual drops by this factor (default 0.1) */
    int poll;           /* iterations between host checks of the device flags (0: automatic) */
    int verify;         /* nonzero: recompute every shifted residual in FP64 at the end (stats) and, in
                           multishift_solve and multishift_bicgstab, refine each system still above
                           tol (see there) */
    int basis_slots;    /* Krylov-basis storage of the non-seed shifts (see multishift_solve):
                           0: automatic (up to half of the device memory free at the start),
                           > 0: at most this many stored residual vectors, < 0: never */
    int graph;          /* 0: the iterations between two polls are captured once as a HIP graph and
                           replayed (not while profiling); < 0: plain launches */
} sgn_ms_opts;

/* BiCG-LR(m) (section "Two-sided Lanczos with rational functions"): for each
 * problem, x_P = R sign(Lambda) L^H b, r = (I - P) b, y = c H_W(mu) r, and the
 * BiCG iterates of all shifted systems (c^2 H_W^2 - sigma_i) x_i = y from one
 * two-sided Lanczos sequence (seed: the shift of smallest modulus; the others
 * by the collinearity of their residuals), x = x_P + sum_i omega_i x_i.
 * Problems may live on different lattices.  stats: nprob entries or NULL.
 * Unless per-shift solutions are requested (x_shift or verify), the non-seed
 * shifts keep no vectors of their own: the seed residuals r_k are stored (they
 * span the Krylov space every p_i and x_i lives in) and sum_{i != seed} omega_i x_i
 * is formed once at the end from the scalar recurrences -- the same iterates,
 * with one stored vector per iteration instead of a read-modify-write of every
 * p_i.  If the stored basis would exceed basis_slots vectors the solver turns
 * the basis into explicit p_i, x_i and continues with per-shift vectors.
 * With LR deflation the exact x_i lie in range(I - P); the components along the
 * deflated eigenvectors that rounding leaves (which the bi-Lanczos process,
 * whose shadow space is orthogonal to them, never reduces) are projected out of
 * the seed solution at every reliable update and out of the combined result at
 * the end, and the mixed schedule stops at FP32 (FP16 links would perturb the
 * operator enough to excite those modes every iteration).
 * With o->verify the per-shift solutions are kept explicitly, every shifted
 * residual y - (c^2 H^2 - sigma_i) x_i is recomputed in FP64 at the end, and each
 * system still above tol gets an FP64 correction before the combination: x_i += e
 * with (c^2 H^2 - sigma_i) e = r_i solved by single-shift FP64 BiCGStab to tol/2
 * (stats: refine_iterations, matvecs; shift_residual holds the final FP64 residuals;
 * SGN_ERR_NOT_CONVERGED if a system stays above tol).
 * Synchronises `stream`.  Returns SGN_ERR_NOT_CONVERGED (x holds the last
 * iterate) if maxiter is reached, SGN_ERR_BREAKDOWN on a BiCG breakdown. */
sgn_status multishift_solve(const sgn_problem *pb, int nprob, const sgn_rational *r, const sgn_ms_opts *o,
                            sgn_stats *stats, void *stream);

/* Multishift BiCGStab (the BiCGStab variant named beside BiCG-LR in the section
 * "Two-sided Lanczos with rational functions"): the same problems, rational
 * function and result as multishift_solve, but every iteration applies
 * c^2 H_W(mu)^2 - sigma_seed twice (to p and to s = r - alpha v) and never the
 * adjoint.  Seed: the shift of smallest modulus, shadow y; the other shifts reuse
 * BiCG's collinearity factors times the stabilising factors prod (1 + omega tau_i).
 * Default form: the seed's r_k and s_k are stored (two vectors per iteration, in
 * the iteration's precision) and sum_{i != seed} omega_i x_i is one lift at the end;
 * scalars stay on the device, the iterations between two polls (o->poll, default 4)
 * are captured once as a HIP graph (o->graph < 0: plain launches), and o->prec,
 * theta32, theta16 and delta give the mixed schedule of multishift_solve (FP64 ->
 * FP32 -> FP16 links, FP64 reliable updates of the seed; FP32 at most with
 * deflation); requested x_i are lifted one by one at the end.  If o->basis_slots < 0,
 * every shift keeps p_i, x_i instead (FP64 only, scalars on the host, three
 * synchronisations per iteration).
 * Slots first written in the FP32 phase hold FP32 vectors.  o->basis_slots > 0 caps the
 * stored bytes at that many FP64 vectors (an FP32 slot counts half; SGN_ERR_NOMEM beyond
 * it; 0: up to half of the free memory).  Only the seed is reliable-updated: in the mixed
 * schedule the other shifted solutions can stay above tol (measured up to 6e-8 relative at
 * 24^3 x 48 with tol 1e-9) although their combination meets it.  With o->verify (stored-basis
 * form) every x_i is lifted explicitly, its residual y - (c^2 H^2 - sigma_i) x_i recomputed in
 * FP64, each system above tol refined by single-shift FP64 BiCGStab to tol/2 as in
 * multishift_solve, and x = x_P + sum_i omega_i x_i formed from the checked x_i (one lift and
 * two FP64 stencil applications per shift; SGN_ERR_NOT_CONVERGED if a system stays above tol).
 * stats: iterations, matvecs, reliable_updates, refine_iterations, shift_residual (collinear
 * estimates, or with verify the FP64 residuals), residual.  Several problems (stored-basis form)
 * run in lockstep: one launch per step of the iteration for all of them (their stencils grouped by
 * lattice into multi-RHS launches, the vector updates and scalar steps over every problem at once,
 * per precision phase), a chunk of o->poll iterations captured once as a HIP graph; each problem
 * has its own reliable updates, precision switches and convergence.  Synchronises `stream`.  SGN_ERR_NOT_CONVERGED after maxiter
 * (x holds the last iterate), SGN_ERR_BREAKDOWN if r^^H r or r^^H v vanishes. */
sgn_status multishift_bicgstab(const sgn_problem *pb, int nprob, const sgn_rational *r, const sgn_ms_opts *o,
                               sgn_stats *stats, void *stream);

/* Multishift QMR (the QMR variant named beside BiCG in the section "Two-sided
 * Lanczos with rational functions"; shifted QMR after Freund): the same problems,
 * rational function and result as multishift_solve.  One two-sided Lanczos
 * sequence on A' = c^2 H_W(mu)^2 (v_1 = y/||y||, shadow w_1 = v_1; four stencil
 * applications per step, two with mu and two with -mu) serves every shift: with
 * A' V_k = V_{k+1} Tbar_k, the iterate of shift i is x_i = V_k z_i where z_i
 * minimises || ||y|| e_1 - (Tbar_k - sigma_i Ibar_k) z ||_2 (Givens QR on the
 * host, one column per step).  Converged when that quasi-residual tau_i is at
 * most tol ||y|| for every shift (checked every o->poll steps, default 4); the
 * true residual is at most ||V_{k+1}||_2 tau_i <= sqrt(k+1) tau_i.  Every basis
 * vector is stored (FP64, pooled in the context between calls; o->basis_slots > 0
 * caps them, 0: up to half of the free device memory, SGN_ERR_NOMEM beyond the
 * cap, < 0 is invalid) and x = x_P + V_k sum_i omega_i z_i is one lift at the
 * end; requested x_i are lifted one by one.  With LR deflation the Krylov part
 * of x and of each x_i is projected with (I - P) at the end.  o->prec: SGN_PREC_F64,
 * or the mixed schedule SGN_PREC_F32: FP64 steps while the largest tau_i is above
 * theta32 ||y||, then the stencil in FP32 (SGN_PREC_F32_H16: and with FP16 links
 * below theta16 ||y||); the recurrences, coefficients and basis stay FP64.  There
 * are no reliable updates: the stencil's rounding enters the Lanczos relation
 * weighted by the size of the late coefficients, which shrink with tau, so the
 * thresholds set the accuracy.  delta is ignored.  stats: iterations, matvecs,
 * shift_residual (tau_i / ||y||; with o->verify the FP64 true residuals), residual,
 * krylov_ms, small_ms (Givens updates).  Several problems run in lockstep: per step
 * one launch for all of them of each stencil application (grouped by lattice into
 * multi-RHS launches), of the update and of the two scalar steps, the step index
 * kept on the device; a chunk of o->poll steps is captured once as a HIP graph
 * (o->graph is ignored) and replayed until a problem changes precision or a quarter
 * of the launch has converged.  Synchronises `stream`.  SGN_ERR_NOT_CONVERGED after
 * maxiter (x holds the last iterate), SGN_ERR_BREAKDOWN on a Lanczos breakdown
 * (w^^H v vanishing; for a batch, the whole call). */
sgn_status multishift_qmr(const sgn_problem *pb, int nprob, const sgn_rational *r, const sgn_ms_opts *o,
                          sgn_stats *stats, void *stream);

/* ------------------------------------------------------------------ accuracy measure */
/* Accuracy of an approximate sign function S (numerical-results section): as
 * sign(A)^2 = I, the value 1/2 ||S(S b) - b|| / ||b|| estimates the error of S
 * without knowing sign(A) b.  The caller applies the same S twice (any of the
 * three methods above, identical options) and passes b and ssb = S(S b), both
 * device canonical complex128 on `lat` (12 V entries).  *acc (host) receives the
 * value; both norms are FP64 sums in a fixed order (deterministic).
 * Synchronises `stream`.  SGN_ERR_INVALID if ||b|| = 0 or a pointer is NULL. */
sgn_status sgn_accuracy_measure(sgn_lattice lat, const void *b, const void *ssb, double *acc, void *stream);

/* ------------------------------------------------------------------ profiling */
/* Per-kernel-class timing of the library's own launches, measured with HIP
 * events on the launch stream, together with the algorithmic HBM bytes (every
 * input read once, every output written once; a link counts as its nine
 * complex entries even where only two rows are stored) and flops of each
 * launch, and the bytes of the stored format.  Meant for roofline reporting.
 * Where a profiled launch is one kernel (the stencil, the BiCGStab and Lanczos
 * vector updates) the kernel's dispatch stamps the event pair with its own
 * start and end (hipExtLaunchKernel), so the time is the kernel's execution;
 * the other classes (multishift updates and lifts, which may span several
 * kernels) are bracketed by event markers, which add a few microseconds of
 * queue latency per launch.  HIP-graph replay is off while profiling. */
typedef enum {
    SGN_K_STENCIL_F64 = 0,
    SGN_K_STENCIL_F32 = 1,
    SGN_K_STENCIL_H16 = 2,
    SGN_K_SHIFT_UPDATE = 3,   /* multishift: x_i += alpha_i p_i, p_i = zeta_i r + beta_i p_i (seed only
                                 when the basis is stored); BiCGStab: the seed's x and p */
    SGN_K_SEED_UPDATE = 4,    /* multishift: r, r~ updates with their inner products; BiCGStab: s = r -
                                 alpha v, the t^H s, t^H t dots, r' = s - omega t with its dots; QMR:
                                 the Lanczos update of v and w with their inner products */
    SGN_K_LIFT = 5,           /* multishift: sum of the stored vectors with their coefficients */
    SGN_K_COUNT = 6
} sgn_kernel_class;

typedef struct {
    long long launches;   /* launches recorded (every N-th one, see sgn_profile_enable) */
    double total_ms;      /* time, bytes and flops of the recorded launches */
    double bytes;
    double flops;
    long long calls;      /* all launches of the class while profiling was on */
    double bytes_stored;  /* bytes of the recorded launches in the stored format (two-row links) */
} sgn_kernel_profile;

/* enable != 0 starts (and resets) profiling on this context; 0 stops it.
 * enable = N > 1 records only every N-th launch of each kernel class (the
 * per-launch averages stay representative while the event markers of the
 * marker-bracketed classes cost 1/N as much). */
sgn_status sgn_profile_enable(sgn_handle h, int enable);
/* Waits for the recorded launches and fills out[SGN_K_COUNT]. */
sgn_status sgn_profile_read(sgn_handle h, sgn_kernel_profile *out);

#ifdef __cplusplus
}
#endif
#endif /* SGN_H */
