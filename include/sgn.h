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
/* Create a context on HIP device `device`.  Owns workspaces and the per-shape
 * launch-configuration cache.  Not thread-safe: use one context per thread. */
sgn_status sgn_init(sgn_handle *h, int device);
sgn_status sgn_finalize(sgn_handle h);
const char *sgn_status_string(sgn_status s);
const char *sgn_last_error(void);

/* ------------------------------------------------------------------ lattice */
/* Pack the gauge field `links` (device, canonical layout, complex128) into the
 * library's internal copies.  `prec_mask` is a bit mask of (1 << sgn_prec)
 * values saying which link precisions to keep (0 = all).  The caller may free
 * `links` once the call returns (the call synchronises `stream`). */
sgn_status sgn_lattice_create(sgn_handle h, const sgn_lattice_desc *d, const void *links,
                              unsigned prec_mask, void *stream, sgn_lattice *out);
sgn_status sgn_lattice_destroy(sgn_lattice lat);
/* sites V and bytes of one spinor in the internal layout for precision p */
int64_t sgn_lattice_volume(sgn_lattice lat);
size_t sgn_spinor_bytes(sgn_lattice lat, sgn_prec p);

/* Canonical <-> internal layout.  `canon` is complex128 for SGN_PREC_F64 and
 * complex64 otherwise; `internal` holds sgn_spinor_bytes(lat, p) bytes. */
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

#ifdef __cplusplus
}
#endif
#endif /* SGN_H */
