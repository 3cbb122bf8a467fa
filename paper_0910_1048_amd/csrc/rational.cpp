// Neuberger rational approximation of sign and the choice of its parameters
// (section "Choice of the rational function": Eqs. (neuberger_mit_c), (pfe_s),
// the circle theorem and Eq. (no_of_poles); spectral-circle heuristic of the
// numerical-results section).
#include <cmath>

#include "sgn_internal.h"

using namespace sgn;

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
