"""Pins of the oracle's sign-function routines and Krylov algorithms.

Each routine is checked against something other than itself: textbook closed
forms of sign for triangular and diagonal matrices, the Hermitian special
case, an independent dense route, exactness of the Krylov methods when the
Krylov space is the whole space, and the identities stated in the paper for
the Neuberger approximation (PFE = closed form, g(1/t) = g(t), the tanh form,
the circle theorem).
"""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, dense, krylov, rational

from conftest import rel


# ----------------------------------------------------------------------------- dense sign
@pytest.mark.parametrize("a,bb", [(0.7 + 0.2j, 1.5 - 0.3j), (2.0, -4.0), (0.1 - 0.05j, 3.0j)])
def test_sign_of_2x2_triangular_closed_form(a, bb):
    """sign([[a, b], [0, -a]]) = [[1, b/a], [0, -1]] for Re a > 0."""
    A = np.array([[a, bb], [0, -a]], dtype=np.complex128)
    want = np.array([[1, bb / a], [0, -1]], dtype=np.complex128)
    for j in range(2):
        e = np.eye(2, dtype=np.complex128)[:, j]
        assert np.allclose(dense.sign_eig(A, e), want[:, j], atol=1e-13)
        assert np.allclose(dense.sign_schur(A, e), want[:, j], atol=1e-13)


def test_sign_of_diagonalisable_with_known_basis(rng):
    lam = np.array([2.0, -1.0 + 0.5j, 0.3 - 2j, -0.2 - 0.1j, 1.1 + 3j])
    R = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    A = R @ np.diag(lam) @ np.linalg.inv(R)
    S = R @ np.diag(np.sign(lam.real)) @ np.linalg.inv(R)
    b = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    assert rel(dense.sign_eig(A, b), S @ b) < 1e-12
    assert rel(dense.sign_schur(A, b), S @ b) < 1e-12


def test_dense_sign_identities_on_lattice():
    dims = (2, 2, 2, 4)
    W = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    A = W.dense(0.3)
    S = dense.sign_schur_matrix(A)
    n = A.shape[0]
    assert np.abs(S @ S - np.eye(n)).max() < 1e-11
    assert np.abs(S @ A - A @ S).max() < 1e-11
    b = synth.gaussian_source(dims, 0).ravel()
    assert rel(dense.sign_eig(A, b), S @ b) < 1e-11


def test_dense_sign_hermitian_case():
    dims = (2, 2, 2, 4)
    W = WilsonRef(synth.gauge_field(dims, 0.5, 3), dims, 0.2)
    A = W.dense(0.0)
    b = synth.gaussian_source(dims, 3).ravel()
    assert rel(dense.sign_eig(A, b), dense.sign_herm(A, b)) < 1e-12
    assert rel(dense.sign_schur(A, b), dense.sign_herm(A, b)) < 1e-12


def test_imaginary_axis_is_rejected():
    A = np.diag([1.0, 1j, -2.0]).astype(np.complex128)
    with pytest.raises(dense.ImaginaryAxisError):
        dense.sign_eig(A, np.ones(3, dtype=np.complex128))


# ----------------------------------------------------------------------------- rational
@pytest.mark.parametrize("s", [8, 10, 16, 70])
def test_pfe_equals_closed_form(s, rng):
    t = (rng.standard_normal(200) + 1j * rng.standard_normal(200)) * 2
    t = t[np.abs(t.real) > 0.05]
    assert np.abs(rational.g_pfe(s, t) - rational.g_closed(s, t)).max() < 1e-12


def test_neuberger_identities(rng):
    s = 12
    t = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    assert np.abs(rational.g_closed(s, 1 / t) - rational.g_closed(s, t)).max() < 1e-12
    assert abs(rational.g_closed(s, 1.0) - 1) < 1e-15
    u = rng.uniform(-0.95, 0.95, 50)
    assert np.abs(rational.g_closed(s, u) - np.tanh(2 * s * np.arctanh(u))).max() < 1e-12
    om, sg = rational.neuberger_pfe(s)
    assert np.all(sg < 0) and np.all(om > 0)


@pytest.mark.parametrize("s,eps", [(8, 1e-4), (16, 1e-8), (30, 1e-12)])
def test_circle_theorem(s, eps):
    M, R = rational.circle(s, eps)
    assert abs(1 + R * R - M * M) < 1e-9 * M * M          # the proof's identity
    th = np.linspace(0, 2 * np.pi, 721)
    for rad in (R, 0.5 * R, 0.999 * R):
        t = M + rad * np.exp(1j * th)
        err = np.abs(rational.g_closed(s, t) - 1.0)
        assert err.max() <= eps + 1e-14          # bound attained to rounding on the circle
    # on the circle boundary the bound is nearly attained somewhere
    t = M + R * np.exp(1j * th)
    assert np.abs(rational.g_closed(s, t) - 1.0).max() > 0.3 * eps
    # mirror circle in the left half plane
    assert np.abs(rational.g_closed(s, -(M + R * np.exp(1j * th))) + 1.0).max() <= eps + 1e-14


@pytest.mark.parametrize("alpha,beta,eps", [(0.2, 2.5, 1e-8), (0.05, 2.6, 1e-8), (0.3, 1.0, 1e-12)])
def test_pole_count_gives_accuracy_on_spectral_circles(alpha, beta, eps):
    s = rational.poles_needed(alpha, beta, eps)
    om, sg, c = rational.coefficients(s, alpha, beta)
    m, r = rational.circle_from_extremes(alpha, beta)
    th = np.linspace(0, 2 * np.pi, 721)
    for rad in (r, 0.7 * r, 0.2 * r):
        t = m + rad * np.exp(1j * th)
        assert np.abs(rational.g_closed(s, c * t) - 1).max() <= eps + 1e-14
    # scaled interval maps to [1/d, d]
    _, d = rational.scale_from_circle(m, r)
    assert abs(c * alpha - 1 / d) < 1e-14 and abs(c * beta - d) < 1e-12


def test_rational_dense_against_eigen_route(rng):
    n = 12
    lam = np.concatenate([rng.uniform(0.3, 2, 6), -rng.uniform(0.3, 2, 6)]) + 0.1j * rng.standard_normal(n)
    R = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = R @ np.diag(lam) @ np.linalg.inv(R)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    s = 10
    om, sg, c = rational.coefficients(s, 0.3, 2.0)
    want = R @ (rational.g_closed(s, c * lam) * np.linalg.solve(R, b))
    assert rel(dense.rational_dense(A, b, om, sg, c), want) < 1e-11


# ----------------------------------------------------------------------------- Krylov
def _small_nonhermitian(rng, n=24):
    lam = np.concatenate([rng.uniform(0.5, 2, n // 2), -rng.uniform(0.5, 2, n - n // 2)])
    lam = lam + 0.2j * rng.standard_normal(n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return Q @ (np.diag(lam) + 0.1 * np.triu(rng.standard_normal((n, n)), 1)) @ Q.conj().T


def test_two_sided_lanczos_exact_on_full_space(rng):
    A = _small_nonhermitian(rng)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x = krylov.lanczos_sign(lambda v: A @ v, lambda v: A.conj().T @ v, b, A.shape[0])
    assert rel(x, dense.sign_schur(A, b)) < 1e-8


def test_two_sided_lanczos_relations(rng):
    """A V = V T + h v e^T and W^H V = I on the first steps; at mu = 0 W = V."""
    dims = (2, 2, 2, 4)
    W_ = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    b = synth.gaussian_source(dims, 0).ravel()
    for mu in (0.3, 0.0):
        A = lambda v: W_.apply(v, mu)
        Ah = lambda v: W_.apply_adj(v, mu)
        x, parts = krylov.lanczos_sign(A, Ah, b, 12, return_parts=True)
        V, Wb, T = parts["V"], parts["W"], parts["T"]
        assert np.abs(Wb.conj() @ V.T - np.eye(12)).max() < 1e-10
        # column j (< k-1) of A V = V T exactly
        for j in range(10):
            lhs = A(V[j])
            rhs = T[:, j] @ V
            assert rel(lhs, rhs) < 1e-12
        if mu == 0.0:
            assert np.abs(Wb - V).max() < 1e-12
            assert np.abs(T - T.conj().T).max() < 1e-12


def test_lanczos_with_full_deflation_is_exact(rng):
    """m = n: x_P alone is sign(A) b and the Krylov part vanishes."""
    A = _small_nonhermitian(rng, 10)
    lam, R = np.linalg.eig(A)
    L = np.linalg.inv(R).conj().T         # L^H R = I
    b = rng.standard_normal(10) + 1j * rng.standard_normal(10)
    xP = krylov.deflation_xP(L, R, lam, b)
    assert rel(xP, dense.sign_schur(A, b)) < 1e-12
    Pb = R @ (L.conj().T @ b)
    assert np.linalg.norm(krylov.project_out(L, R, b)) < 1e-12 * np.linalg.norm(b)
    assert rel(R @ (L.conj().T @ Pb), Pb) < 1e-12  # P^2 = P


def _lattice_deflation(H, m):
    lam, R = np.linalg.eig(H)
    Linv = np.linalg.inv(R)
    idx = np.argsort(np.abs(lam.real))[:m]       # closest to the imaginary axis
    return Linv[idx].conj().T, R[:, idx], lam[idx]


def test_deflated_lanczos_and_rational_against_dense():
    dims = (2, 2, 2, 4)
    W_ = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    mu = 0.3
    H = W_.dense(mu)
    b = synth.gaussian_source(dims, 0).ravel()
    A = lambda v: W_.apply(v, mu)
    Ah = lambda v: W_.apply_adj(v, mu)
    L, R, lam = _lattice_deflation(H, 8)
    assert np.abs(L.conj().T @ R - np.eye(8)).max() < 1e-10
    exact = dense.sign_schur(H, b)
    x = krylov.lanczos_sign(A, Ah, b, 300, L=L, R=R, lam=lam)
    assert rel(x, exact) < 1e-9
    # deflation accelerates the direct method at equal k
    x0 = krylov.lanczos_sign(A, Ah, b, 200)
    x1 = krylov.lanczos_sign(A, Ah, b, 200, L=L, R=R, lam=lam)
    assert rel(x1, exact) < 0.1 * rel(x0, exact)
    ev = np.linalg.eigvals(H)
    rest = np.sort(np.abs(ev))
    alpha = np.min(np.abs(np.setdiff1d(ev, lam)))  # smallest non-deflated modulus
    beta = rest[-1]
    s = rational.poles_needed(alpha, beta, 1e-10)
    om, sg, c = rational.coefficients(s, alpha, beta)
    # the exact rational target with deflation: x_P + g(cA)(I-P)b
    target = krylov.deflation_xP(L, R, lam, b) + dense.rational_dense(H, krylov.project_out(L, R, b), om, sg, c)
    xf = krylov.fom_rational(A, b, om, sg, c, 20, tol=1e-13, L=L, R=R, lam=lam)
    xm = krylov.multishift_bicg(A, Ah, b, om, sg, c, tol=1e-13, L=L, R=R, lam=lam)
    assert rel(xf, target) < 1e-10
    assert rel(xm, target) < 1e-10
    assert rel(target, exact) < 2e-9


def test_rational_krylov_exact_on_small_matrix(rng):
    A = _small_nonhermitian(rng, 20)
    b = rng.standard_normal(20) + 1j * rng.standard_normal(20)
    om, sg, c = rational.coefficients(12, 0.5, 2.1)
    want = dense.rational_dense(A, b, om, sg, c)
    xf = krylov.fom_rational(lambda v: A @ v, b, om, sg, c, 7, tol=1e-13)
    xm = krylov.multishift_bicg(lambda v: A @ v, lambda v: A.conj().T @ v, b, om, sg, c, tol=1e-13)
    assert rel(xf, want) < 1e-11
    assert rel(xm, want) < 1e-10


def test_multishift_shifted_iterates_solve_their_systems(rng):
    """Every shifted iterate x_i satisfies its own system (A' - sigma_i) x_i = y."""
    A = _small_nonhermitian(rng, 30)
    b = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    om, sg, c = rational.coefficients(8, 0.5, 2.1)
    _, info = krylov.multishift_bicg(lambda v: A @ v, lambda v: A.conj().T @ v, b, om, sg, c,
                                     tol=1e-13, return_info=True)
    Ap = c * c * (A @ A)
    y = c * (A @ b)
    for i, s in enumerate(sg):
        assert np.linalg.norm(y - (Ap - s * np.eye(30)) @ info["X"][i]) < 1e-11 * np.linalg.norm(y)


def test_accuracy_measure():
    dims = (2, 2, 2, 4)
    W_ = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    H = W_.dense(0.3)
    S = dense.sign_schur_matrix(H)
    b = synth.gaussian_source(dims, 0).ravel()
    assert krylov.accuracy_measure(lambda v: S @ v, b) < 1e-12
    assert krylov.accuracy_measure(lambda v: 0.99 * (S @ v), b) > 5e-3


def test_restarted_gmres_rational(rng):
    """Restarted GMRES-LR: the dense rational target; the shifted residuals stay
    collinear with the seed's (r_i = rho_i r_seed) after every restart; the seed's
    first-cycle residual is no larger than FOM's (minimal residual over the same
    Krylov space); one cycle with k = n is exact."""
    A = _small_nonhermitian(rng, 30)
    b = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    om, sg, c = rational.coefficients(8, 0.5, 2.1)
    want = dense.rational_dense(A, b, om, sg, c)
    x, info = krylov.gmres_rational(lambda v: A @ v, b, om, sg, c, 6, tol=1e-13, return_info=True)
    assert rel(x, want) < 1e-10
    assert info["cycles"] > 3
    Ap = c * c * (A @ A)
    y = c * (A @ b)
    r_seed = y - (Ap - sg[info["seed"]] * np.eye(30)) @ info["X"][info["seed"]]
    for i, s in enumerate(sg):
        ri = y - (Ap - s * np.eye(30)) @ info["X"][i]
        assert np.linalg.norm(ri - info["rho"][i] * r_seed) <= 1e-10 * np.linalg.norm(y)
    # one cycle each: GMRES seed residual <= FOM seed residual
    _, ig = krylov.gmres_rational(lambda v: A @ v, b, om, sg, c, 5, max_cycles=1, return_info=True)
    _, inf = krylov.fom_rational(lambda v: A @ v, b, om, sg, c, 5, max_cycles=1, return_info=True)
    seed = ig["seed"]
    assert ig["seed_res"][0] <= abs(inf["rho"][seed]) * ig["ynorm"] * (1 + 1e-12)
    # Krylov space of full dimension: exact after one cycle
    x1 = krylov.gmres_rational(lambda v: A @ v, b, om, sg, c, 30, max_cycles=1)
    assert rel(x1, want) < 1e-9


def test_deflated_gmres_rational():
    dims = (2, 2, 2, 4)
    W_ = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    mu = 0.3
    H = W_.dense(mu)
    b = synth.gaussian_source(dims, 0).ravel()
    A = lambda v: W_.apply(v, mu)
    L, R, lam = _lattice_deflation(H, 8)
    ev = np.linalg.eigvals(H)
    alpha = np.min(np.abs(np.setdiff1d(ev, lam)))
    beta = np.max(np.abs(ev))
    om, sg, c = rational.coefficients(12, alpha, beta)
    target = krylov.deflation_xP(L, R, lam, b) + dense.rational_dense(H, krylov.project_out(L, R, b), om, sg, c)
    xg = krylov.gmres_rational(A, b, om, sg, c, 15, tol=1e-13, L=L, R=R, lam=lam)
    assert rel(xg, target) < 1e-10


def test_multishift_bicgstab_shifted_iterates_solve_their_systems(rng):
    """Multishift BiCGStab: every shifted iterate solves its own system (true residual,
    not the collinear estimate), the result equals the dense rational target, and the
    reported shifted residuals are the true ones."""
    n = 40
    A = _small_nonhermitian(rng, n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    om, sg, c = rational.coefficients(8, 0.5, 2.1)
    x, info = krylov.multishift_bicgstab(lambda v: A @ v, b, om, sg, c, tol=1e-12, return_info=True)
    want = dense.rational_dense(A, b, om, sg, c)
    assert rel(x, want) < 1e-9
    Ap = c * c * (A @ A)
    y = info["y"]
    for i, s in enumerate(sg):
        ri = y - (Ap - s * np.eye(n)) @ info["X"][i]
        assert np.linalg.norm(ri) <= 1e-10 * np.linalg.norm(y)
    # stopped early: the seed's collinear estimate is its true residual, and every frozen
    # shift stopped below the tolerance
    x2, info2 = krylov.multishift_bicgstab(lambda v: A @ v, b, om, sg, c, tol=1e-4, return_info=True)
    for i, s in enumerate(sg):
        ri = np.linalg.norm(y - (Ap - s * np.eye(n)) @ info2["X"][i]) / np.linalg.norm(y)
        assert ri <= 1.0001e-4
        if i == info2["seed"]:
            assert ri == pytest.approx(info2["res"][i], rel=1e-6)


def test_deflated_multishift_bicgstab():
    dims = (2, 2, 2, 4)
    W_ = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    mu = 0.3
    H = W_.dense(mu)
    b = synth.gaussian_source(dims, 0).ravel()
    L, R, lam = _lattice_deflation(H, 8)
    ev = np.linalg.eigvals(H)
    alpha = np.min(np.abs(np.setdiff1d(ev, lam)))
    beta = np.max(np.abs(ev))
    om, sg, c = rational.coefficients(12, alpha, beta)
    target = krylov.deflation_xP(L, R, lam, b) + dense.rational_dense(H, krylov.project_out(L, R, b), om, sg, c)
    x = krylov.multishift_bicgstab(lambda v: W_.apply(v, mu), b, om, sg, c, tol=1e-12, L=L, R=R, lam=lam)
    assert rel(x, target) < 1e-9
