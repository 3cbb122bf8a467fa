// sign(T) e_1 for the small projected matrix of the direct two-sided Lanczos
// method (section "Short recurrences": f(H_k) of the k x k projected matrix,
// computed here through its eigendecomposition; the O(k^3) last term of the
// cost proposition of the direct method, which dominates at small volumes).
//
// Route: complex Schur form T = Z S Z^H by the implicit single-shift QR
// algorithm on the (tridiagonal, hence Hessenberg) input; eigenvectors of the
// triangular S by back substitution; then
//   sign(T) e_1 = Z X sign(Lambda) X^{-1} Z^H e_1,
// where X (unit upper triangular) holds the eigenvectors of S.  Z is never
// formed: the QR sweeps record their rotations, and Z^H e_1 and Z u are two
// replays of them (O(1) per rotation instead of a length-k column update).
// The sweeps work on separate real and imaginary planes, apply the column part
// of each rotation along rows after the sweep wherever the sweep no longer reads
// it, and are built for AVX2/FMA as well as for the baseline x86-64 set.
#include "small_sign.h"
#include "sgn_internal.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <limits>
#include <memory>
#include <string>
#include <vector>

namespace sgn {

using zc = std::complex<double>;

namespace {

struct Mat {
    int n;
    std::vector<zc> a;  // row-major
    explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, zc(0, 0)) {}
    zc &operator()(int i, int j) { return a[(size_t)i * n + j]; }
    zc operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

inline double cabs1(zc z) { return std::abs(z.real()) + std::abs(z.imag()); }

// Complex product written out: std::complex's operator* goes through a library
// routine that handles infinities and NaNs, several times slower in these loops
// (all values here are finite).
inline zc cmul(zc a, zc b)
{
    return zc(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}

// Givens (c real, s complex) with G [x; y] = [r; 0], G = [[c, s], [-conj(s), c]].
inline void givens(zc x, zc y, double &c, zc &s)
{
    const double ax = std::abs(x), ay = std::abs(y);
    if (ay == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (ax == 0.0) {
        c = 0.0;
        s = std::conj(y) / ay;
        return;
    }
    const double nrm = std::hypot(ax, ay);
    c = ax / nrm;
    s = (x / ax) * std::conj(y) / nrm;
}

// One plane rotation of the QR sweeps: columns m, m+1 of Z are replaced by
// (c Z_m + conj(s) Z_{m+1}, -s Z_m + c Z_{m+1}), i.e. Z <- Z G with
// G = [c, -s; conj(s), c] on (m, m+1).
struct Rot {
    int m;
    double c;
    zc s;
};

// The sweep kernels are inlined into two builds of the Schur routine (below).
#define SGN_INLINE inline __attribute__((always_inline))

// A square matrix as two row-major planes (real and imaginary parts): the rotation
// loops of the QR sweeps then run on plain double arrays, which the compiler vectorises.
struct Planes {
    int n;
    std::vector<double> re, im;
    explicit Planes(const Mat &A) : n(A.n), re((size_t)A.n * A.n), im((size_t)A.n * A.n)
    {
        for (size_t q = 0; q < A.a.size(); ++q) {
            re[q] = A.a[q].real();
            im[q] = A.a[q].imag();
        }
    }
    zc get(int i, int j) const { return zc(re[(size_t)i * n + j], im[(size_t)i * n + j]); }
    void set(int i, int j, zc v)
    {
        re[(size_t)i * n + j] = v.real();
        im[(size_t)i * n + j] = v.imag();
    }
    double *rr(int i) { return re.data() + (size_t)i * n; }
    double *ri(int i) { return im.data() + (size_t)i * n; }
    void store(Mat &A) const
    {
        for (size_t q = 0; q < A.a.size(); ++q) A.a[q] = zc(re[q], im[q]);
    }
};

// Rows a, b <- G [a; b] over len entries, G = [[c, s], [-conj(s), c]].
SGN_INLINE void rotate_row_pair(double *__restrict ar, double *__restrict ai, double *__restrict br,
                            double *__restrict bi, int len, double c, double sr, double si)
{
    for (int j = 0; j < len; ++j) {
        const double xr = ar[j], xi = ai[j], yr = br[j], yi = bi[j];
        ar[j] = c * xr + sr * yr - si * yi;
        ai[j] = c * xi + sr * yi + si * yr;
        br[j] = c * yr - sr * xr - si * xi;
        bi[j] = c * yi - sr * xi + si * xr;
    }
}

// Rotations of one sweep from the right, applied along R rows at once: for q = 0..cnt-1 in order,
// (row[m], row[m+1]) <- (row[m] c + row[m+1] conj(s), row[m+1] c - row[m] s) with m = m0 + q and
// (c, s) = (gc[q], gsr[q] + i gsi[q]).  The entry moving right is carried in registers (each entry
// is read and written once); the R rows are independent chains, interleaved for the pipelines.
template <int R>
SGN_INLINE void rotate_rows_right(double *const *re, double *const *im, const double *gc, const double *gsr,
                              const double *gsi, int m0, int cnt)
{
    if (cnt <= 0) return;
    double tr[R], ti[R];
    for (int r = 0; r < R; ++r) {
        tr[r] = re[r][m0];
        ti[r] = im[r][m0];
    }
    for (int q = 0; q < cnt; ++q) {
        const double c = gc[q], sr = gsr[q], si = gsi[q];
        const int m = m0 + q;
        for (int r = 0; r < R; ++r) {
            const double yr = re[r][m + 1], yi = im[r][m + 1];
            re[r][m] = c * tr[r] + sr * yr + si * yi;
            im[r][m] = c * ti[r] + sr * yi - si * yr;
            const double nr = c * yr - sr * tr[r] + si * ti[r];
            const double ni = c * yi - sr * ti[r] - si * tr[r];
            tr[r] = nr;
            ti[r] = ni;
        }
    }
    for (int r = 0; r < R; ++r) {
        re[r][m0 + cnt] = tr[r];
        im[r][m0 + cnt] = ti[r];
    }
}

// The sweep's rotations m = max(l, i) .. ihi-1 on rows i = i0 .. i1-1 of P (row i is touched by
// rotation m only if i <= m + 2; rows i <= m are the ones left for after the sweep).
SGN_INLINE void rotate_rows_after_sweep(Planes &P, int i0, int i1, int l, int ihi, const std::vector<double> &gc,
                             const std::vector<double> &gsr, const std::vector<double> &gsi)
{
    constexpr int R = 4;
    int i = i0;
    for (; i + R <= i1; i += R) {
        // rows i..i+R-1 start at max(l, row); bring the earlier ones up to the last row's start
        const int mc = std::max(l, i + R - 1);
        for (int r = 0; r < R - 1; ++r) {
            const int m0 = std::max(l, i + r);
            double *pr[1] = {P.rr(i + r)}, *pi[1] = {P.ri(i + r)};
            rotate_rows_right<1>(pr, pi, gc.data() + (m0 - l), gsr.data() + (m0 - l), gsi.data() + (m0 - l), m0,
                                 std::min(mc, ihi) - m0);
        }
        if (mc >= ihi) continue;
        double *pr[R], *pi[R];
        for (int r = 0; r < R; ++r) {
            pr[r] = P.rr(i + r);
            pi[r] = P.ri(i + r);
        }
        rotate_rows_right<R>(pr, pi, gc.data() + (mc - l), gsr.data() + (mc - l), gsi.data() + (mc - l), mc,
                             ihi - mc);
    }
    for (; i < i1; ++i) {
        const int m0 = std::max(l, i);
        double *pr[1] = {P.rr(i)}, *pi[1] = {P.ri(i)};
        rotate_rows_right<1>(pr, pi, gc.data() + (m0 - l), gsr.data() + (m0 - l), gsi.data() + (m0 - l), m0,
                             ihi - m0);
    }
}

// Complex Schur decomposition of upper Hessenberg H (overwritten by S).  The unitary
// factor is accumulated into *Z, or, with Z null, its rotations are appended to *rots
// (Z = G_1 G_2 ... in that order).  Returns false if the iteration did not converge.
//
// Within a sweep, rotation m acts on rows m, m+1 (from the left) and on columns m, m+1
// (from the right).  Its column part is needed at once only on rows m+1 and m+2, which
// the next rotation reads; rows 0..m are touched by no later row rotation of the sweep,
// so their column rotations are applied after the sweep, along the rows (contiguous in
// the row-major storage) instead of down the columns.
SGN_INLINE bool hessenberg_schur_body(Mat &Hm, Mat *Zm, std::vector<Rot> *rots)
{
    const int n = Hm.n;
    Planes H(Hm);
    std::unique_ptr<Planes> Z(Zm ? new Planes(*Zm) : nullptr);
    const double ulp = std::numeric_limits<double>::epsilon();
    const double smallnum = std::numeric_limits<double>::min() * (n / ulp);
    int ihi = n - 1;
    int its = 0, total = 0;
    const int max_total = 60 * std::max(n, 10);
    std::vector<double> gc, gsr, gsi;
    gc.reserve(n);
    gsr.reserve(n);
    gsi.reserve(n);
    while (ihi >= 0) {
        // look for a negligible subdiagonal entry
        int l = ihi;
        for (; l > 0; --l) {
            const double tst = cabs1(H.get(l - 1, l - 1)) + cabs1(H.get(l, l));
            if (cabs1(H.get(l, l - 1)) <= std::max(ulp * tst, smallnum)) {
                H.set(l, l - 1, 0.0);
                break;
            }
        }
        if (l == ihi) {  // 1x1 block converged
            --ihi;
            its = 0;
            continue;
        }
        if (++total > max_total) return false;
        ++its;
        // shift
        zc sigma;
        if (its % 11 == 10) {  // exceptional shift
            sigma = H.get(ihi, ihi) + 0.75 * std::abs(H.get(ihi, ihi - 1).real());
        } else {
            const zc a = H.get(ihi - 1, ihi - 1), b = H.get(ihi - 1, ihi), c = H.get(ihi, ihi - 1),
                     d = H.get(ihi, ihi);
            const zc tr2 = 0.5 * (a + d);
            const zc disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
            const zc e1 = tr2 + disc, e2 = tr2 - disc;
            sigma = (std::abs(e1 - d) <= std::abs(e2 - d)) ? e1 : e2;
        }
        // implicit single-shift QR sweep on rows/columns l..ihi
        gc.clear();
        gsr.clear();
        gsi.clear();
        for (int m = l; m < ihi; ++m) {
            zc x, y;
            if (m == l) {
                x = H.get(l, l) - sigma;
                y = H.get(l + 1, l);
            } else {
                x = H.get(m, m - 1);
                y = H.get(m + 1, m - 1);
            }
            double c;
            zc s;
            givens(x, y, c, s);
            // rows m, m+1  (all columns from the bulge column to the end: full Schur form)
            const int j0 = (m == l ? l : m - 1);
            rotate_row_pair(H.rr(m) + j0, H.ri(m) + j0, H.rr(m + 1) + j0, H.ri(m + 1) + j0, n - j0, c, s.real(),
                            s.imag());
            if (m > l) H.set(m + 1, m - 1, 0.0);
            // columns m, m+1 on rows m+1, m+2 now; rows 0..m after the sweep
            const int imax = std::min(m + 2, ihi);
            for (int i = m + 1; i <= imax; ++i) {
                const zc t1 = H.get(i, m), t2 = H.get(i, m + 1);
                H.set(i, m, t1 * c + cmul(t2, std::conj(s)));
                H.set(i, m + 1, t2 * c - cmul(t1, s));
            }
            gc.push_back(c);
            gsr.push_back(s.real());
            gsi.push_back(s.imag());
            if (rots) rots->push_back({m, c, s});
        }
        rotate_rows_after_sweep(H, 0, ihi, l, ihi, gc, gsr, gsi);
        if (Z) {
            // every row of Z takes every rotation of the sweep
            constexpr int R = 4;
            int i = 0;
            for (; i + R <= n; i += R) {
                double *pr[R], *pi[R];
                for (int r = 0; r < R; ++r) {
                    pr[r] = Z->rr(i + r);
                    pi[r] = Z->ri(i + r);
                }
                rotate_rows_right<R>(pr, pi, gc.data(), gsr.data(), gsi.data(), l, ihi - l);
            }
            for (; i < n; ++i) {
                double *pr[1] = {Z->rr(i)}, *pi[1] = {Z->ri(i)};
                rotate_rows_right<1>(pr, pi, gc.data(), gsr.data(), gsi.data(), l, ihi - l);
            }
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) H.set(i, j, 0.0);
    H.store(Hm);
    if (Z) Z->store(*Zm);
    return true;
}

// The same routine built for x86-64 with AVX2 and FMA and for the baseline instruction set,
// chosen once from the host's CPU features (SGN_HOST_ISA=baseline in the environment forces
// the baseline build).
__attribute__((target("avx2,fma"))) bool hessenberg_schur_avx2(Mat &H, Mat *Z, std::vector<Rot> *rots)
{
    return hessenberg_schur_body(H, Z, rots);
}

bool hessenberg_schur_base(Mat &H, Mat *Z, std::vector<Rot> *rots) { return hessenberg_schur_body(H, Z, rots); }

bool hessenberg_schur(Mat &H, Mat *Z, std::vector<Rot> *rots)
{
    static const bool avx2 = [] {
        const char *isa = std::getenv("SGN_HOST_ISA");
        if (isa && std::string(isa) == "baseline") return false;
        return __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
    }();
    return avx2 ? hessenberg_schur_avx2(H, Z, rots) : hessenberg_schur_base(H, Z, rots);
}

}  // namespace

int small_sign_e1(int k, const std::complex<double> *diag, const std::complex<double> *sub,
                  const std::complex<double> *sup, std::complex<double> *y, SmallSignInfo *info)
{
    if (k <= 0) return 1;
    Mat S(k);
    double tnorm = 0.0;
    for (int i = 0; i < k; ++i) {
        S(i, i) = diag[i];
        if (i + 1 < k) {
            S(i + 1, i) = sub[i];
            S(i, i + 1) = sup[i];
        }
    }
    for (int i = 0; i < k; ++i) {
        double row = std::abs(diag[i]);
        if (i + 1 < k) row += std::abs(sup[i]);
        if (i > 0) row += std::abs(sub[i - 1]);
        tnorm = std::max(tnorm, row);
    }
    std::vector<Rot> rots;
    if (!hessenberg_schur(S, nullptr, &rots)) return 2;
    // eigenvalues and the imaginary-axis check
    double minre = std::numeric_limits<double>::infinity();
    std::vector<double> sgn(k);
    for (int i = 0; i < k; ++i) {
        const double re = S(i, i).real();
        minre = std::min(minre, std::abs(re));
        sgn[i] = re > 0 ? 1.0 : -1.0;
    }
    if (info) {
        info->min_abs_re = minre;
        info->norm = tnorm;
    }
    if (!(minre > 1e-12 * tnorm)) return 3;
    // eigenvectors of S: column i of X with X(i, i) = 1, X(j > i, i) = 0, built in a
    // contiguous vector (the sums run along rows of S) and kept as row i of Xt = X^T
    const double ulp = std::numeric_limits<double>::epsilon();
    const double smin = std::max(ulp * tnorm, std::numeric_limits<double>::min());
    Mat Xt(k);
    std::vector<zc> xv(k);
    double cond_est = 1.0;
    for (int i = 0; i < k; ++i) {
        xv[i] = 1.0;
        const zc lam = S(i, i);
        for (int j = i - 1; j >= 0; --j) {
            const zc *srow = &S(j, 0);
            double ar = 0.0, ai = 0.0;
            for (int l = j + 1; l <= i; ++l) {
                ar += srow[l].real() * xv[l].real() - srow[l].imag() * xv[l].imag();
                ai += srow[l].real() * xv[l].imag() + srow[l].imag() * xv[l].real();
            }
            zc den = S(j, j) - lam;
            if (std::abs(den) < smin) den = smin;
            xv[j] = -zc(ar, ai) / den;
        }
        double cn = 0.0;
        for (int j = 0; j <= i; ++j) {
            cn += std::norm(xv[j]);
            Xt(i, j) = xv[j];
        }
        cond_est = std::max(cond_est, std::sqrt(cn));
    }
    if (info) info->eigvec_growth = cond_est;
    // q = Z^H e_1 (the first row of Z: e_1^T G_1 G_2 ..., conjugated);
    // c = X^{-1} q (unit upper triangular, solved column by column: rows of Xt)
    std::vector<zc> c(k, zc(0.0, 0.0));
    c[0] = 1.0;
    for (const Rot &g : rots) {
        const zc t1 = c[g.m], t2 = c[g.m + 1];
        c[g.m] = t1 * g.c + t2 * std::conj(g.s);
        c[g.m + 1] = -t1 * g.s + t2 * g.c;
    }
    for (int i = 0; i < k; ++i) c[i] = std::conj(c[i]);
    for (int j = k - 1; j > 0; --j) {
        const zc cj = c[j];
        const zc *xrow = &Xt(j, 0);
        for (int i = 0; i < j; ++i) c[i] -= cmul(xrow[i], cj);
    }
    // u = X sign(Lambda) c ; y = Z u
    std::vector<zc> u(k, zc(0, 0));
    for (int j = 0; j < k; ++j) {
        const zc cj = sgn[j] * c[j];
        const zc *xrow = &Xt(j, 0);
        for (int i = 0; i <= j; ++i) u[i] += cmul(xrow[i], cj);
    }
    // y = Z u = G_1 (G_2 (... u)): the rotations in reverse order
    for (auto it = rots.rbegin(); it != rots.rend(); ++it) {
        const zc t1 = u[it->m], t2 = u[it->m + 1];
        u[it->m] = it->c * t1 - it->s * t2;
        u[it->m + 1] = std::conj(it->s) * t1 + it->c * t2;
    }
    for (int i = 0; i < k; ++i) y[i] = u[i];
    return 0;
}

int small_eig(int n, const std::complex<double> *a, std::complex<double> *lam, std::complex<double> *vec)
{
    if (n <= 0) return 1;
    Mat H(n), Z(n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) H(i, j) = a[(size_t)i * n + j];
    for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
    // Householder reduction to upper Hessenberg form, H = Z^H A Z
    for (int k = 0; k + 2 < n; ++k) {
        double xn = 0.0;
        for (int i = k + 1; i < n; ++i) xn += std::norm(H(i, k));
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const zc x0 = H(k + 1, k);
        const zc ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : zc(1.0, 0.0);
        std::vector<zc> v(n, zc(0, 0));
        for (int i = k + 1; i < n; ++i) v[i] = H(i, k);
        v[k + 1] += ph * xn;  // v = x + e^{i arg x0} ||x|| e_1: no cancellation
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
        vn = std::sqrt(vn);
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        for (int j = 0; j < n; ++j) {  // H = (I - 2 v v^H) H
            zc d = 0.0;
            for (int i = k + 1; i < n; ++i) d += std::conj(v[i]) * H(i, j);
            for (int i = k + 1; i < n; ++i) H(i, j) -= 2.0 * v[i] * d;
        }
        for (int i = 0; i < n; ++i) {  // H = H (I - 2 v v^H), Z = Z (I - 2 v v^H)
            zc d = 0.0, e = 0.0;
            for (int j = k + 1; j < n; ++j) {
                d += H(i, j) * v[j];
                e += Z(i, j) * v[j];
            }
            for (int j = k + 1; j < n; ++j) {
                H(i, j) -= 2.0 * d * std::conj(v[j]);
                Z(i, j) -= 2.0 * e * std::conj(v[j]);
            }
        }
        for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
    }
    if (!hessenberg_schur(H, &Z, nullptr)) return 2;
    double tnorm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) tnorm = std::max(tnorm, std::abs(H(i, j)));
    const double smin = std::max(std::numeric_limits<double>::epsilon() * tnorm, std::numeric_limits<double>::min());
    for (int i = 0; i < n; ++i) {
        lam[i] = H(i, i);
        // eigenvector of the triangular factor, X(i) = 1, back substitution above it
        std::vector<zc> x(n, zc(0, 0));
        x[i] = 1.0;
        for (int j = i - 1; j >= 0; --j) {
            zc acc = 0.0;
            for (int l = j + 1; l <= i; ++l) acc += H(j, l) * x[l];
            zc den = H(j, j) - lam[i];
            if (std::abs(den) < smin) den = smin;
            x[j] = -acc / den;
        }
        double nrm = 0.0;
        std::vector<zc> u(n, zc(0, 0));
        for (int r = 0; r < n; ++r) {
            for (int l = 0; l <= i; ++l) u[r] += Z(r, l) * x[l];
            nrm += std::norm(u[r]);
        }
        nrm = std::sqrt(nrm);
        for (int r = 0; r < n; ++r) vec[(size_t)r * n + i] = u[r] / nrm;
    }
    return 0;
}

}  // namespace sgn

extern "C" sgn_status sgn_small_sign(int k, const double *diag, const double *sub, const double *sup, double *y,
                                     double *min_abs_re)
{
    using zc = std::complex<double>;
    return sgn::guard([&] {
        SGN_REQUIRE(k >= 1 && diag && y && (k == 1 || (sub && sup)), "sgn_small_sign: bad arguments");
        for (int i = 0; i < 2 * k; ++i) SGN_REQUIRE(std::isfinite(diag[i]), "sgn_small_sign: diag not finite");
        for (int i = 0; i < 2 * (k - 1); ++i)
            SGN_REQUIRE(std::isfinite(sub[i]) && std::isfinite(sup[i]), "sgn_small_sign: sub/sup not finite");
        sgn::SmallSignInfo info;
        const int rc = sgn::small_sign_e1(k, reinterpret_cast<const zc *>(diag), reinterpret_cast<const zc *>(sub),
                                          reinterpret_cast<const zc *>(sup), reinterpret_cast<zc *>(y), &info);
        if (rc == 3) throw sgn::Failure{SGN_ERR_IMAG_AXIS, "sgn_small_sign: eigenvalue on the imaginary axis"};
        if (rc != 0) throw sgn::Failure{SGN_ERR_BREAKDOWN, "sgn_small_sign: QR iteration did not converge"};
        if (min_abs_re) *min_abs_re = info.min_abs_re;
    });
}
