// Host-code exercise under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).
//
// Drives the library's host-only parts -- the small sign of the direct Lanczos method, the small
// general eigensolver, the rational coefficient routines -- and the oracle's C Wilson operator over
// edge and ordinary sizes; any out-of-bounds access, use after free, leak or undefined operation
// aborts the run.  Light result checks keep the calls meaningful: sign(T) e_1 is finite (or the
// imaginary-axis status), A v = lambda v for the eigenpairs, the Neuberger weights are positive,
// and the oracle's adjoint is the adjoint of its operator.
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "sgn.h"
#include "small_sign.h"

namespace sgn {
void set_error(const std::string &) {}  // the library's per-thread message store is not linked here
}

extern "C" {
void oracle_dirac(const double *U, const double *in, double *out, const int *L, double kappa, double mu,
                  const double *bf, const double *bb, int g5);
void oracle_dirac_adj(const double *U, const double *in, double *out, const int *L, double kappa, double mu,
                      const double *bf, const double *bb, int g5, double *scratch);
}

using cd = std::complex<double>;
static int failures = 0;
#define CHECK(c, ...)                          \
    do {                                       \
        if (!(c)) {                            \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");        \
            ++failures;                        \
        }                                      \
    } while (0)

int main()
{
    std::mt19937_64 rng(7);
    std::normal_distribution<double> g(0.0, 1.0);
    // small sign of random tridiagonal matrices (a Lanczos-like spectrum on both sides of the axis)
    for (int k : {1, 2, 3, 7, 50, 200}) {
        std::vector<cd> d(k), sb(k), sp(k), y(k);
        for (int i = 0; i < k; ++i) {
            d[i] = cd((i % 2 ? -1.0 : 1.0) * (0.5 + std::abs(g(rng))), 0.1 * g(rng));
            sb[i] = cd(0.3 * g(rng), 0.1 * g(rng));
            sp[i] = cd(0.3 * g(rng), 0.1 * g(rng));
        }
        sgn::SmallSignInfo info;
        const int rc = sgn::small_sign_e1(k, d.data(), sb.data(), sp.data(), y.data(), &info);
        CHECK(rc == 0 || rc == 3, "small_sign_e1 k=%d returned %d", k, rc);
        if (rc == 0)
            for (int i = 0; i < k; ++i) CHECK(std::isfinite(std::abs(y[i])), "small_sign_e1 k=%d: y not finite", k);
        std::vector<double> yr(2 * k);
        const sgn_status st = sgn_small_sign(k, reinterpret_cast<const double *>(d.data()),
                                             reinterpret_cast<const double *>(sb.data()),
                                             reinterpret_cast<const double *>(sp.data()), yr.data(), nullptr);
        CHECK(st == SGN_OK || st == SGN_ERR_IMAG_AXIS, "sgn_small_sign k=%d status %d", k, (int)st);
    }
    {  // refusals
        cd one(1.0, 0.0);
        double y[2];
        CHECK(sgn_small_sign(0, nullptr, nullptr, nullptr, y, nullptr) != SGN_OK, "k = 0 accepted");
        (void)one;
    }
    // small general eigenproblems
    for (int n : {1, 2, 5, 40}) {
        std::vector<cd> a((size_t)n * n), lam(n), v((size_t)n * n);
        for (auto &e : a) e = cd(g(rng), g(rng));
        const int rc = sgn::small_eig(n, a.data(), lam.data(), v.data());
        CHECK(rc == 0, "small_eig n=%d returned %d", n, rc);
        double worst = 0.0;
        for (int j = 0; j < n && rc == 0; ++j) {
            double r = 0.0;
            for (int i = 0; i < n; ++i) {
                cd acc = 0.0;
                for (int l = 0; l < n; ++l) acc += a[(size_t)i * n + l] * v[(size_t)l * n + j];
                r += std::norm(acc - lam[j] * v[(size_t)i * n + j]);
            }
            worst = std::max(worst, std::sqrt(r) / std::max(std::abs(lam[j]), 1.0));
        }
        CHECK(worst < 1e-10, "small_eig n=%d residual %.3e", n, worst);
    }
    // rational coefficients
    for (int s : {1, 8, 16, 64}) {
        sgn_rational r{};
        CHECK(sgn_rational_neuberger(s, 0.12, 2.6, &r) == SGN_OK, "neuberger s=%d", s);
        for (int i = 0; i < s; ++i) CHECK(r.omega[i] > 0 && r.sigma[i] < 0, "neuberger s=%d coefficient %d", s, i);
        double err = 0.0;
        CHECK(sgn_rational_neuberger_rescaled(s, 0.12, 2.6, &r, &err) == SGN_OK, "rescaled s=%d", s);
        CHECK(sgn_rational_zolotarev(s, 0.12, 2.6, &r, &err) == SGN_OK, "zolotarev s=%d", s);
    }
    {
        int s = 0;
        CHECK(sgn_poles_needed(0.12, 2.6, 1e-8, &s) == SGN_OK && s > 0, "poles_needed");
        sgn_rational r{};
        CHECK(sgn_rational_neuberger(SGN_MAX_POLES + 1, 0.12, 2.6, &r) != SGN_OK, "too many poles accepted");
        CHECK(sgn_rational_neuberger(4, 2.6, 0.12, &r) != SGN_OK, "alpha > beta accepted");
    }
    // the oracle's operator and its adjoint on a 4x4x4x6 lattice of random (not unitary) links
    {
        const int L[4] = {4, 4, 4, 6};
        const int V = L[0] * L[1] * L[2] * L[3];
        std::vector<cd> U((size_t)V * 4 * 9), x((size_t)V * 12), y((size_t)V * 12), hx((size_t)V * 12),
            hy((size_t)V * 12), scratch((size_t)V * 12);
        for (auto &e : U) e = cd(g(rng), g(rng));
        for (auto &e : x) e = cd(g(rng), g(rng));
        for (auto &e : y) e = cd(g(rng), g(rng));
        const double bf[8] = {1, 0, 1, 0, 1, 0, -1, 0}, bb[8] = {1, 0, 1, 0, 1, 0, -1, 0};
        const double *u = reinterpret_cast<const double *>(U.data());
        oracle_dirac(u, reinterpret_cast<const double *>(x.data()), reinterpret_cast<double *>(hx.data()), L, 0.2, 0.3,
                     bf, bb, 1);
        oracle_dirac_adj(u, reinterpret_cast<const double *>(y.data()), reinterpret_cast<double *>(hy.data()), L, 0.2,
                         0.3, bf, bb, 1, reinterpret_cast<double *>(scratch.data()));
        cd a = 0.0, b = 0.0;
        for (size_t i = 0; i < x.size(); ++i) {
            a += std::conj(y[i]) * hx[i];
            b += std::conj(hy[i]) * x[i];
        }
        CHECK(std::abs(a - b) <= 1e-12 * std::abs(a), "oracle adjoint mismatch %.3e", std::abs(a - b));
    }
    std::printf("host sanitizer run: %d failures\n", failures);
    return failures ? 1 : 0;
}
