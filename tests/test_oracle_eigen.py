"""Pins of the oracle's critical eigenpairs (LR deflation).

The eigenpairs come from a dense eigendecomposition; they are checked against
what fixes them independently: the eigen-relations and biorthonormality, the
free-field spectrum in closed form, and the projector onto the critical
invariant subspace built from ordered Schur forms of A and A^H (a different
factorisation, unique for a cut at a gap).
"""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import WilsonRef, eigen

from conftest import rel


def _schur_projector(A, cut):
    """Oblique projector onto the right invariant subspace of the eigenvalues with
    |Re lambda| < cut, along the complement of the matching left subspace."""
    T, Q, k = scipy.linalg.schur(A, output="complex", sort=lambda z: abs(z.real) < cut)
    Tl, W, kl = scipy.linalg.schur(A.conj().T, output="complex", sort=lambda z: abs(z.real) < cut)
    assert k == kl
    Qr, Wl = Q[:, :k], W[:, :k]
    return Qr @ np.linalg.solve(Wl.conj().T @ Qr, Wl.conj().T), k


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_relations_and_schur_projector(mu):
    dims = (2, 2, 2, 4)
    H = WilsonRef(synth.gauge_field(dims, 0.5, 0), dims, 0.2).dense(mu)
    b = synth.gaussian_source(dims, 0).ravel()
    ev = np.sort(np.abs(np.linalg.eigvals(H).real))
    m = int(np.argmax(ev[5:24] / ev[4:23])) + 5  # cut at the widest relative gap, 5..23 vectors
    L, R, lam = eigen.critical_eigenpairs(H, m)
    assert np.abs(H @ R - R * lam).max() < 1e-12
    assert np.abs(L.conj().T @ H - lam[:, None] * L.conj().T).max() < 1e-11
    assert np.abs(L.conj().T @ R - np.eye(m)).max() < 1e-11
    assert np.allclose(np.linalg.norm(R, axis=0), 1.0)
    assert np.allclose(np.sort(np.abs(lam.real)), ev[:m], rtol=1e-12)
    P, k = _schur_projector(H, 0.5 * (ev[m - 1] + ev[m]))
    assert k == m
    assert rel(eigen.projector_apply(L, R, b), P @ b) < 1e-10


def _free_field_eigenvalues(dims, kappa, mu):
    """+-sqrt(M(q)^2 + sum_nu s_nu(q)^2) per momentum, 6-fold each (spin x colour)."""
    out = []
    for a in range(dims[0]):
        for b in range(dims[1]):
            for c in range(dims[2]):
                for d in range(dims[3]):
                    q = np.array([2 * np.pi * a / dims[0], 2 * np.pi * b / dims[1], 2 * np.pi * c / dims[2],
                                  2 * np.pi * (d + 0.5) / dims[3]], dtype=np.complex128)
                    q[3] += 1j * mu
                    lam = np.sqrt((1 - 2 * kappa * np.cos(q).sum()) ** 2 + ((2 * kappa * np.sin(q)) ** 2).sum())
                    out += [lam] * 6 + [-lam] * 6
    return np.array(out)


def test_free_field_cluster():
    """Unit links: the eigenvalues come in closed form with 6-fold degeneracy; the
    projector of a whole degenerate cluster is still unique."""
    dims = (2, 2, 2, 4)
    mu = 0.2
    H = WilsonRef(synth.unit_gauge_field(dims), dims, 0.2).dense(mu)
    want = _free_field_eigenvalues(dims, 0.2, mu)
    order = np.argsort(np.abs(want.real), kind="stable")
    lev = np.abs(want.real)[order]
    m = int(np.nonzero(lev[1:] > lev[:-1] * (1 + 1e-9))[0][0]) + 1  # the first whole cluster
    L, R, lam = eigen.critical_eigenpairs(H, m)
    assert np.allclose(np.sort(np.abs(lam.real)), lev[:m], rtol=1e-6)  # degenerate: sqrt(eps) sensitivity
    assert np.abs(L.conj().T @ R - np.eye(m)).max() < 1e-9
    b = synth.gaussian_source(dims, 1).ravel()
    P, k = _schur_projector(H, 0.5 * (lev[m - 1] + lev[m]))
    assert k == m
    assert rel(eigen.projector_apply(L, R, b), P @ b) < 1e-8
