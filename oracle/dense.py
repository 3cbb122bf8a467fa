"""Dense matrix sign on tiny lattices (test infrastructure only).

Three routes to sign(A) b, each from its own definition:
  sign_eig    -- f(A) b = R f(Lambda) R^{-1} b with sign z = sign Re z
                 (introduction, Eqs. (1) and (matfun_action)).
  sign_schur  -- Schur-Sylvester route: A = Z T Z^H with the right-half-plane
                 eigenvalues ordered first; sign(T) = [[I, X], [0, -I]] with
                 T11 X - X T22 = 2 T12.  Independent of eigenvectors.
  sign_herm   -- Hermitian case (mu = 0): A = Q diag(lambda) Q^H.
Plus the exact rational target g_s(cA) b for the rational methods
(section on the choice of the rational function, Eq. (pfe_s)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class ImaginaryAxisError(ValueError):
    """sign is undefined for an eigenvalue on the imaginary axis."""


def _check_axis(lam, A_norm, rel=1e-12):
    if np.min(np.abs(lam.real)) < rel * A_norm:
        raise ImaginaryAxisError("eigenvalue on (or within rounding of) the imaginary axis")


def sign_eig(A, b, return_cond: bool = False):
    """sign(A) b via the eigendecomposition A = R Lambda R^{-1}."""
    lam, R = np.linalg.eig(A)
    _check_axis(lam, np.linalg.norm(A, 2) if A.shape[0] <= 512 else np.abs(A).sum(0).max())
    y = np.linalg.solve(R, b)
    x = R @ (np.sign(lam.real) * y)
    if return_cond:
        return x, np.linalg.cond(R)
    return x


def sign_schur_matrix(A):
    """sign(A) as a dense matrix via the sorted complex Schur form."""
    T, Z, sdim = sla.schur(A, output="complex", sort="rhp")
    lam = np.diag(T)
    _check_axis(lam, np.abs(A).sum(0).max())
    n = A.shape[0]
    k = int(sdim)
    S = np.zeros_like(T)
    S[:k, :k] = np.eye(k)
    S[k:, k:] = -np.eye(n - k)
    if 0 < k < n:
        # T11 X - X T22 = 2 T12   (scipy solves a X + X b = q)
        X = sla.solve_sylvester(T[:k, :k], -T[k:, k:], 2.0 * T[:k, k:])
        S[:k, k:] = X
    return Z @ S @ Z.conj().T


def sign_schur(A, b):
    return sign_schur_matrix(A) @ b


def sign_herm(A, b):
    """Hermitian A: sign(A) b = Q sign(lambda) Q^H b."""
    lam, Q = np.linalg.eigh(A)
    _check_axis(lam.astype(np.complex128), np.max(np.abs(lam)))
    return Q @ (np.sign(lam) * (Q.conj().T @ b))


def rational_dense(A, b, omega, sigma, c):
    """Exact g_s(cA) b = sum_i omega_i (c^2 A^2 - sigma_i)^{-1} (c A b) by dense LU."""
    n = A.shape[0]
    A2 = (c * c) * (A @ A)
    y = c * (A @ b)
    x = np.zeros(n, dtype=np.complex128)
    for w, s in zip(omega, sigma):
        x += w * np.linalg.solve(A2 - s * np.eye(n), y)
    return x
