"""Pins of the oracle's rescaled Neuberger and Zolotarev approximations.

Rescaled Neuberger: the largest real-axis error of g_s(ct) on [alpha, beta] has
the closed form 2q/(1+q), q = ((d-1)/(d+1))^{2s} (g_s is monotone on each side
of 1 and g_s(1/t) = g_s(t)), and the rescaling lowers it to e_max/(2 - e_max).
Zolotarev: the one-pole case against the best approximation worked out by
hand; for more poles the error equioscillates at 2n+1 points of [k, 1] with one
magnitude (the alternation theorem certifies the best approximation of its
type); the partial fractions equal the product form; on a Hermitian lattice
matrix the error of sign(H) b stays within the uniform bound.
"""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, dense, rational

from conftest import rel


def _g_pfe(om, sg, t):
    t = np.asarray(t, dtype=np.complex128)
    return t * sum(w / (t * t - q) for w, q in zip(om, sg))


def _extrema(f):
    """The extreme value of f on every run of samples of one sign (consecutive
    extrema of an equioscillating error lie in consecutive runs)."""
    cut = np.nonzero(np.sign(f[1:]) != np.sign(f[:-1]))[0] + 1
    return np.array([run[np.argmax(np.abs(run))] for run in np.split(f, cut)])


@pytest.mark.parametrize("s,alpha,beta", [(4, 0.1, 2.0), (8, 0.15, 2.6), (16, 0.05, 2.5)])
def test_rescaled_neuberger_error(s, alpha, beta):
    om, sg, c, e_max = rational.neuberger_rescaled(s, alpha, beta)
    d = np.sqrt(beta / alpha)
    q = ((d - 1) / (d + 1)) ** (2 * s)
    assert e_max == pytest.approx(2 * q / (1 + q), rel=1e-9)
    om0, sg0, c0 = rational.coefficients(s, alpha, beta)
    assert c == c0 and np.all(sg == sg0)
    t = np.geomspace(alpha, beta, 100001)
    err = np.abs(_g_pfe(om, sg, c * t).real - 1.0)
    assert err.max() == pytest.approx(e_max / (2 - e_max), rel=1e-7)
    # the plain approximation's error on the same grid is e_max
    assert np.abs(_g_pfe(om0, sg0, c * t).real - 1.0).max() == pytest.approx(e_max, rel=1e-7)


@pytest.mark.parametrize("k", [0.05, 0.3])
def test_zolotarev_one_pole_closed_form(k):
    """n = 1: D t/(t^2 + c) on [k, 1]; equal errors at both ends force c = k, the maximum
    sits at sqrt(k) with value 1/(2 sqrt k), the minimum 1/(1+k) at the ends."""
    om, sg, c, delta = rational.zolotarev(1, k, 1.0)
    assert c == 1.0
    assert sg[0] == pytest.approx(-k, rel=1e-12)
    fmax, fmin = 1 / (2 * np.sqrt(k)), 1 / (1 + k)
    assert om[0] == pytest.approx(2 / (fmax + fmin), rel=1e-10)
    assert delta == pytest.approx((fmax - fmin) / (fmax + fmin), rel=1e-10)


@pytest.mark.parametrize("n,alpha,beta", [(2, 0.1, 2.0), (3, 0.05, 1.0), (5, 0.2, 2.6), (8, 0.1, 2.0)])
def test_zolotarev_equioscillates(n, alpha, beta):
    om, sg, c, delta = rational.zolotarev(n, alpha, beta)
    assert c == pytest.approx(1 / beta)
    assert np.all(sg < 0) and np.all(om > 0)
    t = np.geomspace(alpha, beta, 400001)
    e = _g_pfe(om, sg, c * t).real - 1.0
    ext = _extrema(e)
    assert len(ext) == 2 * n + 1
    assert np.all(np.sign(ext[1:]) == -np.sign(ext[:-1]))  # alternating signs
    assert np.allclose(np.abs(ext), delta, rtol=1e-5)
    assert np.abs(e).max() <= delta * (1 + 1e-9)
    # odd in t: the same on the negative interval
    assert np.allclose(_g_pfe(om, sg, -c * t).real, -_g_pfe(om, sg, c * t).real)


def test_zolotarev_partial_fractions_equal_product(rng):
    n, alpha, beta = 6, 0.12, 2.4
    om, sg, c, delta = rational.zolotarev(n, alpha, beta)
    k = alpha / beta
    z = rng.standard_normal(20) + 1j * rng.standard_normal(20)
    # D from the value at t = beta (x = 1), an error extremum of size delta below 1
    D = (1 - delta) / rational.zolotarev_unscaled(n, k, 1.0).real
    assert np.allclose(_g_pfe(om, sg, z), D * rational.zolotarev_unscaled(n, k, z), rtol=1e-10)


def test_zolotarev_error_decreases_and_beats_neuberger():
    alpha, beta = 0.1, 2.5
    deltas = [rational.zolotarev(n, alpha, beta)[3] for n in (2, 4, 6, 8)]
    assert all(a > 10 * b for a, b in zip(deltas, deltas[1:]))
    # on the real interval, the Neuberger error with as many poles is far larger
    for n, dz in zip((4, 8), deltas[1::2]):
        _, _, _, e_max = rational.neuberger_rescaled(n, alpha, beta)
        assert dz < 0.1 * e_max


def test_zolotarev_sign_of_hermitian_lattice_matrix():
    dims = (2, 2, 2, 4)
    W = WilsonRef(synth.gauge_field(dims, 0.5, 2), dims, 0.2)
    H = W.dense(0.0)
    b = synth.gaussian_source(dims, 2).ravel()
    ev = np.abs(np.linalg.eigvalsh(H))
    alpha, beta = ev.min() * 0.999, ev.max() * 1.001
    want = dense.sign_herm(H, b)
    for n in (4, 8, 12):
        om, sg, c, delta = rational.zolotarev(n, alpha, beta)
        got = dense.rational_dense(H, b, om, sg, c)
        assert rel(got, want) <= delta * (1 + 1e-6)
    assert rel(got, want) < 1e-9
