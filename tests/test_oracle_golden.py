"""The stored 4^4 dense results agree with an independent oracle route (two-sided
Lanczos / restarted FOM), so a stale or corrupted fixture fails here."""
import os

import numpy as np

import synth
from oracle import WilsonRef, dense, krylov, rational

from conftest import rel

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_dense.npz")


def _c1():
    dims = (4, 4, 4, 4)
    W = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    b = synth.gaussian_source(dims, 0).ravel()
    return W, b, np.load(GOLD)


def test_c1_dense_sign_matches_lanczos_route():
    W, b, g = _c1()
    x = krylov.lanczos_sign(lambda v: W.apply(v, 0.3), lambda v: W.apply_adj(v, 0.3), b, 320)
    assert rel(x, g["sign_b"]) < 1e-9


def test_c1_rational_matches_fom_route():
    W, b, g = _c1()
    om, sg, c = rational.coefficients(16, float(g["alpha"]), float(g["beta"]))
    x = krylov.fom_rational(lambda v: W.apply(v, 0.3), b, om, sg, c, 30, tol=1e-13)
    assert rel(x, g["g16_b"]) < 1e-11
    # circle-theorem level agreement of the rational approximation with the sign
    assert rel(g["g16_b"], g["sign_b"]) < 1e-8


def test_unconverged_lanczos_amplifies_rounding():
    """At k = 200 (not converged on the 4^4 configuration) a 1e-15 relative change
    of b moves the two-sided Lanczos result by far more than 1e-15; once converged
    (k = 320) it does not.  This bounds how closely two FP64 implementations can
    agree before convergence."""
    W, b, g = _c1()
    A = lambda v: W.apply(v, 0.3)
    Ah = lambda v: W.apply_adj(v, 0.3)
    bp = b * (1 + 1e-15 * np.random.default_rng(1).standard_normal(b.size))
    d200 = rel(krylov.lanczos_sign(A, Ah, bp, 200), krylov.lanczos_sign(A, Ah, b, 200))
    d320 = rel(krylov.lanczos_sign(A, Ah, bp, 320), krylov.lanczos_sign(A, Ah, b, 320))
    assert 1e-9 < d200 < 3e-7
    assert d320 < 1e-9


def test_accuracy_measure_tracks_the_rational_error():
    # g_16 is a rational function of A, so S = sign(A) + E with E commuting with
    # sign(A) and S^2 - I = 2 sign(A) E + E^2: half the defect of S^2 b is the
    # error of S b to first order (numerical-results section)
    g = np.load(GOLD)
    b = synth.gaussian_source((4, 4, 4, 4), 0).ravel()
    err = np.linalg.norm(g["g16_b"] - g["sign_b"]) / np.linalg.norm(b)
    acc = float(g["acc16"])
    assert 0.5 < acc / err < 2.0
    assert abs(0.5 * np.linalg.norm(g["g16_g16_b"] - b) / np.linalg.norm(b) - acc) < 1e-20
    # the exact sign squares to the identity
    rng = np.random.default_rng(3)
    A = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)) + 3 * np.diag(np.sign(rng.standard_normal(12)))
    v = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    assert krylov.accuracy_measure(lambda w: dense.sign_eig(A, w), v) < 1e-12


def test_c1_deflation_fixture_consistent():
    """The stored deflation data agree with the stored spectrum (the 15 eigenvalues
    closest to the imaginary axis; alpha of the rest) and with an independent
    route: sign(H) b - x_P = sign(H)(I - P) b by the undeflated two-sided Lanczos
    oracle on b - P b, against the stored dense sign(H) b."""
    W, b, g = _c1()
    d = np.load(os.path.join(os.path.dirname(GOLD), "c1_deflation.npz"))
    ev = g["evals"]
    o = np.argsort(np.abs(ev.real))
    assert np.allclose(np.sort(np.abs(d["lam"].real)), np.abs(ev.real)[o[:15]], rtol=1e-10)
    assert abs(d["alpha_rest"] - np.abs(ev[o[15:]]).min()) < 1e-12
    r = b - d["Pb"]
    y = krylov.lanczos_sign(lambda v: W.apply(v, 0.3), lambda v: W.apply_adj(v, 0.3), r, 400)
    assert rel(d["xP"] + y, g["sign_b"]) < 1e-8
