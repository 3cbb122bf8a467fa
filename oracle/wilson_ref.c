/*
 * Plain FP64 CPU reference of the Wilson-Dirac operator at nonzero chemical
 * potential.  TEST INFRASTRUCTURE ONLY: the oracle is called by the tests,
 * by the smoke check and by the benchmark's CPU-baseline leg, never by the
 * product path.  It shares no code with the HIP library.
 *
 * The paper takes the kernel H_W = gamma5 D_W(mu) from its reference on the
 * overlap operator at nonzero chemical potential and does not print D_W
 * (introduction; numerical-results section).  The reading implemented here:
 *
 *   (D_W psi)(x) = psi(x) - kappa * sum_{nu=1..4} [
 *        w^f_nu (1 - gamma_nu) U_nu(x)        psi(x + nu)
 *      + w^b_nu (1 + gamma_nu) U_nu(x - nu)^H psi(x - nu) ]
 *
 * with w^f_4 = exp(-mu), w^b_4 = exp(+mu), spatial weights 1, and a boundary
 * factor on every hop that wraps around the lattice (periodic in space,
 * antiperiodic in time by default).  Gamma matrices: DeGrand-Rossi chiral
 * basis; gamma5 = gamma1 gamma2 gamma3 gamma4 is computed, not typed in.
 *
 * Deliberately naive: every hop applies the full 4x4 spin matrix and the full
 * 3x3 colour matrix; no spin projection.  The adjoint is computed on its own,
 * as the conjugate transpose of every stored hop block (gathered per site), so
 * that the identity D_W(mu)^H = gamma5 D_W(-mu) gamma5 is a test, not an input.
 *
 * Layouts (complex128, interleaved re/im):
 *   links  [t][z][y][x][nu][3][3]  row-major U_nu(x), nu = x,y,z,t
 *   spinor [t][z][y][x][spin][colour]
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static cplx GAM[4][4][4];   /* gamma_1..gamma_4 */
static cplx PF[4][4][4];    /* 1 - gamma_nu (forward hop)  */
static cplx PB[4][4][4];    /* 1 + gamma_nu (backward hop) */
static cplx G5[4][4];       /* gamma1 gamma2 gamma3 gamma4 */
static int g_ready = 0;

static void init_gammas(void)
{
    if (g_ready) return;
    memset(GAM, 0, sizeof GAM);
    /* gamma_1 */
    GAM[0][0][3] = I;  GAM[0][1][2] = I;  GAM[0][2][1] = -I; GAM[0][3][0] = -I;
    /* gamma_2 */
    GAM[1][0][3] = -1; GAM[1][1][2] = 1;  GAM[1][2][1] = 1;  GAM[1][3][0] = -1;
    /* gamma_3 */
    GAM[2][0][2] = I;  GAM[2][1][3] = -I; GAM[2][2][0] = -I; GAM[2][3][1] = I;
    /* gamma_4 */
    GAM[3][0][2] = 1;  GAM[3][1][3] = 1;  GAM[3][2][0] = 1;  GAM[3][3][1] = 1;
    for (int n = 0; n < 4; ++n)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx id = (i == j) ? 1.0 : 0.0;
                PF[n][i][j] = id - GAM[n][i][j];
                PB[n][i][j] = id + GAM[n][i][j];
            }
    /* gamma5 as the ordered product gamma1 gamma2 gamma3 gamma4 */
    cplx a[4][4], b[4][4];
    memcpy(a, GAM[0], sizeof a);
    for (int n = 1; n < 4; ++n) {
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx s = 0;
                for (int k = 0; k < 4; ++k) s += a[i][k] * GAM[n][k][j];
                b[i][j] = s;
            }
        memcpy(a, b, sizeof a);
    }
    memcpy(G5, a, sizeof a);
    g_ready = 1;
}

/* Export the matrices so that the tests can check the Clifford algebra. */
void oracle_gammas(double *out /* 5*4*4 complex */)
{
    init_gammas();
    cplx *o = (cplx *)out;
    for (int n = 0; n < 4; ++n)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) o[(n * 4 + i) * 4 + j] = GAM[n][i][j];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) o[(4 * 4 + i) * 4 + j] = G5[i][j];
}

typedef struct {
    int L[4];
    double kappa, mu;
    cplx bf[4], bb[4]; /* factors on forward / backward hops that wrap */
} geom;

static inline int64_t site_of(const geom *g, const int c[4])
{
    return c[0] + (int64_t)g->L[0] * (c[1] + (int64_t)g->L[1] * (c[2] + (int64_t)g->L[2] * c[3]));
}

static inline void coords_of(const geom *g, int64_t s, int c[4])
{
    c[0] = (int)(s % g->L[0]); s /= g->L[0];
    c[1] = (int)(s % g->L[1]); s /= g->L[1];
    c[2] = (int)(s % g->L[2]); s /= g->L[2];
    c[3] = (int)s;
}

/* neighbour in direction nu, dir=+1 forward, -1 backward; *wrap set if the hop crosses the edge */
static inline int64_t neighbour(const geom *g, const int c[4], int nu, int dir, int *wrap)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[nu] += dir;
    *wrap = 0;
    if (d[nu] >= g->L[nu]) { d[nu] -= g->L[nu]; *wrap = 1; }
    if (d[nu] < 0) { d[nu] += g->L[nu]; *wrap = 1; }
    return site_of(g, d);
}

/* acc += coef * (S or S^H) (x) (C or C^H) v  for a 12-vector v[spin][colour] */
static void block_apply(cplx acc[12], const cplx S[4][4], int s_adj,
                        const cplx *C, int c_adj, cplx coef, const cplx *v)
{
    cplx t[4][3];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx sum = 0;
            for (int b = 0; b < 3; ++b) {
                cplx cab = c_adj ? conj(C[b * 3 + a]) : C[a * 3 + b];
                sum += cab * v[s * 3 + b];
            }
            t[s][a] = sum;
        }
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx sum = 0;
            for (int r = 0; r < 4; ++r) {
                cplx ssr = s_adj ? conj(S[r][s]) : S[s][r];
                sum += ssr * t[r][a];
            }
            acc[s * 3 + a] += coef * sum;
        }
}

/* v <- gamma5 v  (adj != 0: v <- gamma5^H v) */
static void apply_g5(cplx v[12], int adj)
{
    cplx t[12];
    for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) {
            cplx sum = 0;
            for (int r = 0; r < 4; ++r) sum += (adj ? conj(G5[r][s]) : G5[s][r]) * v[r * 3 + a];
            t[s * 3 + a] = sum;
        }
    memcpy(v, t, sizeof t);
}

static inline double w_fwd(const geom *g, int nu) { return nu == 3 ? exp(-g->mu) : 1.0; }
static inline double w_bwd(const geom *g, int nu) { return nu == 3 ? exp(g->mu) : 1.0; }

/* D_W (or gamma5 D_W) at a single site x */
static void dirac_site(const geom *g, const cplx *U, const cplx *in, cplx out[12], int64_t x, int g5)
{
    int c[4];
    coords_of(g, x, c);
    cplx acc[12];
    for (int i = 0; i < 12; ++i) acc[i] = in[x * 12 + i];
    for (int nu = 0; nu < 4; ++nu) {
        int wr;
        int64_t xp = neighbour(g, c, nu, +1, &wr);
        cplx cf = -g->kappa * w_fwd(g, nu) * (wr ? g->bf[nu] : 1.0);
        block_apply(acc, PF[nu], 0, U + (x * 4 + nu) * 9, 0, cf, in + xp * 12);
        int64_t xm = neighbour(g, c, nu, -1, &wr);
        cplx cb = -g->kappa * w_bwd(g, nu) * (wr ? g->bb[nu] : 1.0);
        block_apply(acc, PB[nu], 0, U + (xm * 4 + nu) * 9, 1, cb, in + xm * 12);
    }
    if (g5) apply_g5(acc, 0);
    memcpy(out, acc, sizeof acc);
}

/*
 * Adjoint at site y, from the conjugate transposes of the hop blocks of the
 * sites that reach y: the forward block of x = y - nu (which reads psi(y)) and
 * the backward block of x = y + nu (which reads psi(y)).  For gamma5 D_W the
 * adjoint is D_W^H gamma5^H, so gamma5^H is applied to the input first (the
 * caller passes that product).
 */
static void dirac_adj_site(const geom *g, const cplx *U, const cplx *in, cplx out[12], int64_t y)
{
    int c[4];
    coords_of(g, y, c);
    cplx acc[12];
    for (int i = 0; i < 12; ++i) acc[i] = in[y * 12 + i];
    for (int nu = 0; nu < 4; ++nu) {
        int wr;
        /* x = y - nu; its forward hop x -> x+nu = y wraps iff the backward step from y wraps */
        int64_t x = neighbour(g, c, nu, -1, &wr);
        cplx cf = -g->kappa * w_fwd(g, nu) * (wr ? g->bf[nu] : 1.0);
        block_apply(acc, PF[nu], 1, U + (x * 4 + nu) * 9, 1, conj(cf), in + x * 12);
        /* x = y + nu; its backward hop x -> x-nu = y uses U_nu(x - nu) = U_nu(y) (adjointed in D) */
        x = neighbour(g, c, nu, +1, &wr);
        cplx cb = -g->kappa * w_bwd(g, nu) * (wr ? g->bb[nu] : 1.0);
        block_apply(acc, PB[nu], 1, U + (y * 4 + nu) * 9, 0, conj(cb), in + x * 12);
    }
    memcpy(out, acc, sizeof acc);
}

static void make_geom(geom *g, const int *L, double kappa, double mu, const double *bf, const double *bb)
{
    init_gammas();
    for (int i = 0; i < 4; ++i) {
        g->L[i] = L[i];
        g->bf[i] = bf[2 * i] + I * bf[2 * i + 1];
        g->bb[i] = bb[2 * i] + I * bb[2 * i + 1];
    }
    g->kappa = kappa;
    g->mu = mu;
}

static int64_t volume(const int *L) { return (int64_t)L[0] * L[1] * L[2] * L[3]; }

/* out = D_W(mu) in  (g5 != 0: out = gamma5 D_W(mu) in) */
void oracle_dirac(const double *U, const double *in, double *out, const int *L,
                  double kappa, double mu, const double *bf, const double *bb, int g5)
{
    geom g;
    make_geom(&g, L, kappa, mu, bf, bb);
    const int64_t V = volume(L);
    const cplx *u = (const cplx *)U, *p = (const cplx *)in;
    cplx *o = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < V; ++x) dirac_site(&g, u, p, o + x * 12, x, g5);
}

/* out = D_W(mu)^H in  (g5 != 0: out = (gamma5 D_W(mu))^H in = D_W^H gamma5 in) */
void oracle_dirac_adj(const double *U, const double *in, double *out, const int *L,
                      double kappa, double mu, const double *bf, const double *bb, int g5,
                      double *scratch /* 12 V complex, used when g5 != 0 */)
{
    geom g;
    make_geom(&g, L, kappa, mu, bf, bb);
    const int64_t V = volume(L);
    const cplx *u = (const cplx *)U;
    const cplx *p = (const cplx *)in;
    if (g5) {
        cplx *t = (cplx *)scratch;
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < V; ++x) {
            memcpy(t + x * 12, p + x * 12, 12 * sizeof(cplx));
            apply_g5(t + x * 12, 1);
        }
        p = t;
    }
    cplx *o = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < V; ++y) dirac_adj_site(&g, u, p, o + y * 12, y);
}

/* Forward operator at a list of sites only: out[i] = (D or gamma5 D)(sites[i]) */
void oracle_dirac_sites(const double *U, const double *in, double *out, const int *L,
                        double kappa, double mu, const double *bf, const double *bb, int g5,
                        const int64_t *sites, int64_t nsites)
{
    geom g;
    make_geom(&g, L, kappa, mu, bf, bb);
    const cplx *u = (const cplx *)U, *p = (const cplx *)in;
    cplx *o = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nsites; ++i) dirac_site(&g, u, p, o + i * 12, sites[i], g5);
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
