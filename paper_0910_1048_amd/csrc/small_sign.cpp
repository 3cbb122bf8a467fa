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
#include "small_sign.h"
#include "sgn_internal.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
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

// Complex Schur decomposition of upper Hessenberg H (overwritten by S).  The unitary
// factor is accumulated into *Z, or, with Z null, its rotations are appended to *rots
// (Z = G_1 G_2 ... in that order).  Returns false if the iteration did not converge.
bool hessenberg_schur(Mat &H, Mat *Z, std::vector<Rot> *rots = nullptr)
{
    const int n = H.n;
    const double ulp = std::numeric_limits<double>::epsilon();
    const double smallnum = std::numeric_limits<double>::min() * (n / ulp);
    int ihi = n - 1;
    int its = 0, total = 0;
    const int max_total = 60 * std::max(n, 10);
    while (ihi >= 0) {
        // look for a negligible subdiagonal entry
        int l = ihi;
        for (; l > 0; --l) {
            const double tst = cabs1(H(l - 1, l - 1)) + cabs1(H(l, l));
            if (cabs1(H(l, l - 1)) <= std::max(ulp * tst, smallnum)) {
                H(l, l - 1) = 0.0;
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
            sigma = H(ihi, ihi) + 0.75 * std::abs(H(ihi, ihi - 1).real());
        } else {
            const zc a = H(ihi - 1, ihi - 1), b = H(ihi - 1, ihi), c = H(ihi, ihi - 1), d = H(ihi, ihi);
            const zc tr2 = 0.5 * (a + d);
            const zc disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
            const zc e1 = tr2 + disc, e2 = tr2 - disc;
            sigma = (std::abs(e1 - d) <= std::abs(e2 - d)) ? e1 : e2;
        }
        // implicit single-shift QR sweep on rows/columns l..ihi
        for (int m = l; m < ihi; ++m) {
            zc x, y;
            if (m == l) {
                x = H(l, l) - sigma;
                y = H(l + 1, l);
            } else {
                x = H(m, m - 1);
                y = H(m + 1, m - 1);
            }
            double c;
            zc s;
            givens(x, y, c, s);
            // rows m, m+1  (all columns from the bulge column to the end: full Schur form)
            for (int j = (m == l ? l : m - 1); j < n; ++j) {
                const zc t1 = H(m, j), t2 = H(m + 1, j);
                H(m, j) = c * t1 + cmul(s, t2);
                H(m + 1, j) = c * t2 - cmul(std::conj(s), t1);
            }
            if (m > l) H(m + 1, m - 1) = 0.0;
            // columns m, m+1
            const int imax = std::min(m + 2, ihi);
            for (int i = 0; i <= imax; ++i) {
                const zc t1 = H(i, m), t2 = H(i, m + 1);
                H(i, m) = t1 * c + cmul(t2, std::conj(s));
                H(i, m + 1) = t2 * c - cmul(t1, s);
            }
            if (Z) {
                for (int i = 0; i < n; ++i) {
                    const zc t1 = (*Z)(i, m), t2 = (*Z)(i, m + 1);
                    (*Z)(i, m) = t1 * c + cmul(t2, std::conj(s));
                    (*Z)(i, m + 1) = t2 * c - cmul(t1, s);
                }
            } else {
                rots->push_back({m, c, s});
            }
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) H(i, j) = 0.0;
    return true;
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
    // eigenvectors of S: X(:, i) with X(i, i) = 1, X(j > i, i) = 0
    const double ulp = std::numeric_limits<double>::epsilon();
    const double smin = std::max(ulp * tnorm, std::numeric_limits<double>::min());
    Mat X(k);
    double cond_est = 1.0;
    for (int i = 0; i < k; ++i) {
        X(i, i) = 1.0;
        const zc lam = S(i, i);
        for (int j = i - 1; j >= 0; --j) {
            zc acc = 0.0;
            for (int l = j + 1; l <= i; ++l) acc += cmul(S(j, l), X(l, i));
            zc den = S(j, j) - lam;
            if (std::abs(den) < smin) den = smin;
            X(j, i) = -acc / den;
        }
        double cn = 0.0;
        for (int j = 0; j <= i; ++j) cn += std::norm(X(j, i));
        cond_est = std::max(cond_est, std::sqrt(cn));
    }
    if (info) info->eigvec_growth = cond_est;
    // q = Z^H e_1 (the first row of Z: e_1^T G_1 G_2 ..., conjugated);
    // c = X^{-1} q (unit upper triangular back substitution)
    std::vector<zc> c(k, zc(0.0, 0.0));
    c[0] = 1.0;
    for (const Rot &g : rots) {
        const zc t1 = c[g.m], t2 = c[g.m + 1];
        c[g.m] = t1 * g.c + t2 * std::conj(g.s);
        c[g.m + 1] = -t1 * g.s + t2 * g.c;
    }
    for (int i = 0; i < k; ++i) c[i] = std::conj(c[i]);
    for (int i = k - 1; i >= 0; --i) {
        zc acc = c[i];
        for (int j = i + 1; j < k; ++j) acc -= cmul(X(i, j), c[j]);
        c[i] = acc;
    }
    // u = X sign(Lambda) c ; y = Z u
    std::vector<zc> u(k, zc(0, 0));
    for (int j = 0; j < k; ++j) {
        const zc cj = sgn[j] * c[j];
        for (int i = 0; i <= j; ++i) u[i] += cmul(X(i, j), cj);
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
    if (!hessenberg_schur(H, &Z)) return 2;
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
