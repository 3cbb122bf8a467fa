"""Pins of the oracle's multishift QMR.

The QMR iterates are checked against things other than the routine itself:
the Hermitian case, where two-sided Lanczos is orthonormal and QMR is the
minimal-residual iterate over an explicitly built Krylov basis; exactness when
the Krylov space is the whole space; the identity that ties the quasi-residual
norms tau_k to the residual norms rho_j of the Galerkin (BiCG) iterates of the
same Lanczos sequence, 1/tau_k^2 = sum_{j<=k} 1/rho_j^2, with rho_j taken from
the oracle's independent multishift BiCG; the residual bound
||r|| <= sqrt(k+1) tau; and the dense rational target on a small lattice, with
and without LR deflation.
"""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, dense, krylov, rational

from conftest import rel


def _nonhermitian(rng, n):
    lam = np.concatenate([rng.uniform(0.5, 2, n // 2), -rng.uniform(0.5, 2, n - n // 2)])
    lam = lam + 0.2j * rng.standard_normal(n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return Q @ (np.diag(lam) + 0.1 * np.triu(rng.standard_normal((n, n)), 1)) @ Q.conj().T


def _ops(A):
    return (lambda v: A @ v), (lambda v: A.conj().T @ v)


def test_qmr_hermitian_case_is_minimal_residual(rng):
    """A Hermitian: A' = c^2 A^2 is Hermitian, the Lanczos basis is orthonormal and the
    QMR iterate minimises the true residual over K_k(A', y); compare with that minimum
    over a basis built from the powers A'^j y."""
    n, k = 40, 5
    lam = np.concatenate([rng.uniform(0.3, 2, n // 2), -rng.uniform(0.3, 2, n - n // 2)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    A = Q @ np.diag(lam) @ Q.conj().T
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    om, sg, c = rational.coefficients(6, 0.3, 2.0)
    _, info = krylov.multishift_qmr(*_ops(A), b, om, sg, c, k=k, return_info=True)
    Ap = c * c * (A @ A)
    y = c * (A @ b)
    K = np.empty((n, k), dtype=np.complex128)
    K[:, 0] = y
    for j in range(1, k):
        K[:, j] = Ap @ K[:, j - 1]
    B, _ = np.linalg.qr(K)
    for i, s in enumerate(sg):
        coef = np.linalg.lstsq((Ap - s * np.eye(n)) @ B, y, rcond=None)[0]
        xm = B @ coef
        assert rel(info["X"][i], xm) < 1e-9
        r = np.linalg.norm(y - (Ap - s * np.eye(n)) @ xm)
        assert info["tau"][i] == pytest.approx(r, rel=1e-9)


def test_qmr_exact_on_full_space(rng):
    n = 10
    A = _nonhermitian(rng, n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    om, sg, c = rational.coefficients(5, 0.5, 2.1)
    x, info = krylov.multishift_qmr(*_ops(A), b, om, sg, c, k=n, return_info=True)
    Ap = c * c * (A @ A)
    y = c * (A @ b)
    for i, s in enumerate(sg):
        assert rel(info["X"][i], np.linalg.solve(Ap - s * np.eye(n), y)) < 1e-8
    assert rel(x, dense.rational_dense(A, b, om, sg, c)) < 1e-8


def test_qmr_quasi_residuals_follow_the_bicg_residuals(rng):
    """1/tau_k^2 = sum_{j=0..k} 1/rho_j^2 for every shift, rho_j the residual norm of the
    BiCG iterate after j iterations (rho_0 = ||y||), BiCG run by its own routine.  (Both
    come from the Givens QR of Tbar_k - sigma Ibar_k: tau_k = tau_{k-1} |s_k| and
    rho_k = tau_k / |c_k|; the BiCG residual is h_{k+1,k} |e_k^T z_G| ||v_{k+1}|| with
    ||v_{k+1}|| = 1.)"""
    n, kmax = 60, 10
    A = _nonhermitian(rng, n)
    A_, Ah_ = _ops(A)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    om, sg, c = rational.coefficients(6, 0.5, 2.1)
    Ap = c * c * (A @ A)
    y = c * (A @ b)
    rho = [np.full(len(sg), np.linalg.norm(y))]
    for j in range(1, kmax + 1):
        _, bi = krylov.multishift_bicg(A_, Ah_, b, om, sg, c, tol=1e-300, maxiter=j, return_info=True)
        rho.append(np.array([np.linalg.norm(y - (Ap - s * np.eye(n)) @ bi["X"][i]) for i, s in enumerate(sg)]))
    rho = np.array(rho)
    for k in range(1, kmax + 1):
        _, qi = krylov.multishift_qmr(A_, Ah_, b, om, sg, c, k=k, return_info=True)
        want = 1.0 / np.sqrt(np.sum(1.0 / rho[:k + 1] ** 2, axis=0))
        # rho_j of tiny residuals carry the rounding of forming y - M x (~1e-16 ||y||)
        assert np.allclose(qi["tau"], want, rtol=1e-7, atol=1e-13 * np.linalg.norm(y))


def test_qmr_residual_bound_and_monotone_quasi_residual(rng):
    n = 50
    A = _nonhermitian(rng, n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    om, sg, c = rational.coefficients(6, 0.5, 2.1)
    Ap = c * c * (A @ A)
    prev = None
    for k in (2, 5, 9, 14, 20):
        _, info = krylov.multishift_qmr(*_ops(A), b, om, sg, c, k=k, return_info=True)
        for i, s in enumerate(sg):
            r = np.linalg.norm(info["y"] - (Ap - s * np.eye(n)) @ info["X"][i])
            # slack for the rounding floor of r and tau (~1e-15 ||y||)
            assert r <= np.sqrt(k + 1) * info["tau"][i] * (1 + 1e-10) + 1e-13 * info["ynorm"]
        if prev is not None:
            assert np.all(info["tau"] <= prev * (1 + 1e-12) + 1e-13 * info["ynorm"])
        prev = info["tau"]


def test_qmr_stops_below_tolerance(rng):
    n = 40
    A = _nonhermitian(rng, n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    om, sg, c = rational.coefficients(8, 0.5, 2.1)
    x, info = krylov.multishift_qmr(*_ops(A), b, om, sg, c, tol=1e-11, return_info=True)
    assert np.all(info["tau"] <= 1e-11 * info["ynorm"])
    assert rel(x, dense.rational_dense(A, b, om, sg, c)) < 1e-9


def _lattice_deflation(H, m):
    lam, R = np.linalg.eig(H)
    Linv = np.linalg.inv(R)
    idx = np.argsort(np.abs(lam.real))[:m]
    return Linv[idx].conj().T, R[:, idx], lam[idx]


@pytest.mark.parametrize("m", [0, 8])
def test_qmr_lattice_rational_target(m):
    dims = (2, 2, 2, 4)
    W_ = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2)
    mu = 0.3
    H = W_.dense(mu)
    b = synth.gaussian_source(dims, 0).ravel()
    ev = np.linalg.eigvals(H)
    if m:
        L, R, lam = _lattice_deflation(H, m)
        rest = np.setdiff1d(ev, lam)
    else:
        L = R = lam = None
        rest = ev
    om, sg, c = rational.coefficients(12, np.min(np.abs(rest)), np.max(np.abs(ev)))
    target = krylov.deflation_xP(L, R, lam, b) + dense.rational_dense(H, krylov.project_out(L, R, b), om, sg, c)
    x = krylov.multishift_qmr(lambda v: W_.apply(v, mu), lambda v: W_.apply_adj(v, mu), b, om, sg, c,
                              tol=1e-12, check_every=4, L=L, R=R, lam=lam)
    assert rel(x, target) < 1e-9
