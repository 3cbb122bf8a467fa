// Rational approximations of sign and the choice of their parameters
// (section "Choice of the rational function": Eqs. (neuberger_mit_c), (pfe_s),
// the circle theorem and Eq. (no_of_poles); spectral-circle heuristic of the
// numerical-results section; the rescaled Neuberger function of the footnote
// on the choice of c; Zolotarev's best approximation, named there for spectra
// close to the real axis).
#include <algorithm>
#include <cmath>
#include <vector>

#include "sgn_internal.h"

using namespace sgn;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Arithmetic-geometric mean sequences for parameter m = modulus^2 (descending
// Landen transformation): a_0 = 1, b_0 = sqrt(1-m), c_0 = sqrt(m).
struct Agm {
    std::vector<double> a, c;
};

Agm agm(double m)
{
    Agm g;
    double a = 1.0, b = std::sqrt(1.0 - m), c = std::sqrt(m);
    g.a.push_back(a);
    g.c.push_back(c);
    for (int it = 0; it < 64 && std::abs(c) > 1e-17 * a; ++it) {
        const double an = 0.5 * (a + b), bn = std::sqrt(a * b);
        c = 0.5 * (a - b);
        a = an;
        b = bn;
        g.a.push_back(a);
        g.c.push_back(c);
    }
    return g;
}

// complete elliptic integral of the first kind, K(m) = pi / (2 AGM(1, sqrt(1-m)))
double ellip_k(double m) { return kPi / (2.0 * agm(m).a.back()); }

// Jacobi sn and cn of argument u, parameter m: phi_N = 2^N a_N u, then
// phi_{j-1} = (phi_j + asin(c_j sin(phi_j) / a_j)) / 2 down to phi_0; sn = sin phi_0
void ellip_sncn(double u, double m, double &sn, double &cn)
{
    const Agm g = agm(m);
    const int N = (int)g.a.size() - 1;
    double phi = std::ldexp(g.a[N] * u, N);
    for (int j = N; j >= 1; --j) phi = 0.5 * (phi + std::asin(g.c[j] / g.a[j] * std::sin(phi)));
    sn = std::sin(phi);
    cn = std::cos(phi);
}

// x prod_{l<n} (x^2 + c_{2l}) / prod_{l<=n} (x^2 + c_{2l-1}), cc[l-1] = c_l
double zolo_unscaled(const std::vector<double> &cc, int n, double x)
{
    double v = x;
    const double x2 = x * x;
    for (int l = 1; l < n; ++l) v *= x2 + cc[2 * l - 1];
    for (int l = 1; l <= n; ++l) v /= x2 + cc[2 * l - 2];
    return v;
}

// golden-section search for an extremum of f on [lo, hi] (sgn = +1: maximum)
template <typename F> double golden_extremum(F f, double lo, double hi, double sgn)
{
    const double r = 0.5 * (std::sqrt(5.0) - 1.0);
    double x1 = hi - r * (hi - lo), x2 = lo + r * (hi - lo);
    double f1 = sgn * f(x1), f2 = sgn * f(x2);
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
        if (f1 > f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - r * (hi - lo);
            f1 = sgn * f(x1);
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + r * (hi - lo);
            f2 = sgn * f(x2);
        }
    }
    return sgn * std::max(f1, f2);
}

}  // namespace

extern "C" sgn_status sgn_rational_neuberger(int s, double alpha, double beta, sgn_rational *out)
{
    return guard([&] {
        SGN_REQUIRE(out != nullptr, "sgn_rational_neuberger: null output");
        SGN_REQUIRE(s >= 1 && s <= SGN_MAX_POLES, "sgn_rational_neuberger: s out of range");
        SGN_REQUIRE(std::isfinite(alpha) && std::isfinite(beta) && alpha > 0 && beta > alpha,
                    "sgn_rational_neuberger: need 0 < alpha < beta");
        *out = sgn_rational{};
        out->s = s;
        const double m = 0.5 * (alpha + beta), r = 0.5 * (beta - alpha);
        out->c = 1.0 / std::sqrt((m + r) * (m - r));
        out->alpha = alpha;
        out->beta = beta;
        const double pi = 3.14159265358979323846;
        for (int i = 1; i <= s; ++i) {
            const double th = pi / (2.0 * s) * (i - 0.5);
            const double ct = std::cos(th), tt = std::tan(th);
            out->omega[i - 1] = 1.0 / (s * ct * ct);
            out->sigma[i - 1] = -tt * tt;
        }
    });
}

extern "C" sgn_status sgn_poles_needed(double alpha, double beta, double eps, int *s)
{
    return guard([&] {
        SGN_REQUIRE(s != nullptr, "sgn_poles_needed: null output");
        SGN_REQUIRE(alpha > 0 && beta > alpha && eps > 0 && eps < 1, "sgn_poles_needed: bad arguments");
        const double m = 0.5 * (alpha + beta), r = 0.5 * (beta - alpha);
        const double d = std::sqrt((m + r) / (m - r));
        const double bound = std::log(eps / (eps + 2.0)) / (2.0 * std::log((d - 1.0) / (d + 1.0)));
        *s = (int)std::ceil(bound - 1e-12);
        if (*s < 1) *s = 1;
    });
}

extern "C" sgn_status sgn_rational_neuberger_rescaled(int s, double alpha, double beta, sgn_rational *out, double *err)
{
    sgn_status st = sgn_rational_neuberger(s, alpha, beta, out);
    if (st != SGN_OK) return st;
    return guard([&] {
        // on [alpha, beta] the scaled argument spans [1/d, d], d = sqrt(beta/alpha); g_s is
        // monotone on each side of 1 with g_s(1/t) = g_s(t), so the largest error is at the ends:
        // e_max = 1 - g_s(d) = 2q/(1+q), q = ((d-1)/(d+1))^{2s}; the factor 2/(2 - e_max) = 1 + q
        // turns it into e_max/(2 - e_max) = q
        const double d = std::sqrt(beta / alpha);
        const double q = std::pow((d - 1.0) / (d + 1.0), 2.0 * s);
        for (int i = 0; i < s; ++i) out->omega[i] *= 1.0 + q;
        if (err) *err = q;
    });
}

extern "C" sgn_status sgn_rational_zolotarev(int s, double alpha, double beta, sgn_rational *out, double *err)
{
    return guard([&] {
        SGN_REQUIRE(out != nullptr, "sgn_rational_zolotarev: null output");
        SGN_REQUIRE(s >= 1 && s <= SGN_MAX_POLES, "sgn_rational_zolotarev: s out of range");
        SGN_REQUIRE(std::isfinite(alpha) && std::isfinite(beta) && alpha > 0 && beta > alpha,
                    "sgn_rational_zolotarev: need 0 < alpha < beta");
        const int n = s;
        const double k = alpha / beta, mp = 1.0 - k * k;
        const double Kp = ellip_k(mp);
        std::vector<double> cc(2 * n - 1);
        for (int l = 1; l <= 2 * n - 1; ++l) {
            double sn, cn;
            ellip_sncn(l * Kp / (2.0 * n), mp, sn, cn);
            cc[l - 1] = k * k * sn * sn / (cn * cn);
        }
        // D = 2/(max + min) of the unscaled function on [k, 1]: a log grid, the error of a
        // provisional D split into runs of one sign, the largest deviation of each run
        // refined by golden section (ends included)
        auto f = [&](double x) { return zolo_unscaled(cc, n, x); };
        const int G = 4096 * n;
        std::vector<double> xs(G), fs(G);
        for (int j = 0; j < G; ++j) {
            xs[j] = k * std::pow(1.0 / k, (double)j / (G - 1));
            fs[j] = f(xs[j]);
        }
        const auto mm = std::minmax_element(fs.begin(), fs.end());
        const double D0 = 2.0 / (*mm.first + *mm.second);
        double fmax = std::max(fs[0], fs[G - 1]), fmin = std::min(fs[0], fs[G - 1]);
        for (int lo = 0; lo < G;) {
            const bool above = D0 * fs[lo] > 1.0;
            int hi = lo, jb = lo;
            for (; hi < G && (D0 * fs[hi] > 1.0) == above; ++hi)
                if (std::abs(D0 * fs[hi] - 1.0) > std::abs(D0 * fs[jb] - 1.0)) jb = hi;
            const double a = xs[std::max(jb - 1, 0)], b = xs[std::min(jb + 1, G - 1)];
            if (above)
                fmax = std::max(fmax, golden_extremum(f, a, b, 1.0));
            else
                fmin = std::min(fmin, golden_extremum(f, a, b, -1.0));
            lo = hi;
        }
        const double D = 2.0 / (fmax + fmin);
        *out = sgn_rational{};
        out->s = n;
        out->c = 1.0 / beta;
        out->alpha = alpha;
        out->beta = beta;
        for (int i = 0; i < n; ++i) {  // residues of the product form at x^2 = -c_{2i+1}
            const double ci = cc[2 * i];
            double a = 1.0;
            for (int l = 1; l < n; ++l) a *= cc[2 * l - 1] - ci;
            for (int l = 0; l < n; ++l)
                if (l != i) a /= cc[2 * l] - ci;
            out->omega[i] = D * a;
            out->sigma[i] = -ci;
        }
        if (err) *err = (fmax - fmin) / (fmax + fmin);
    });
}
