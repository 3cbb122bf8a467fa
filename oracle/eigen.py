"""Critical eigenpairs for LR deflation -- TEST INFRASTRUCTURE ONLY.

Section "Deflation": the critical eigenvalues of the sign function are those
closest to the imaginary axis; LR deflation needs their right eigenvectors
R_m (A R_m = R_m Lambda_m) and left eigenvectors L_m (L_m^H A = Lambda_m L_m^H),
normalised to L_m^H R_m = I so that P = R_m L_m^H is a projector.

critical_eigenpairs is that definition written out with a dense
eigendecomposition A = X Lambda X^{-1}: R_m are m columns of X, L_m^H the
matching rows of X^{-1} (biorthonormal by construction, also inside a
degenerate eigenspace).
"""
from __future__ import annotations

import numpy as np


def critical_eigenpairs(A, m: int):
    """(L, R, lam): the m eigenvalues of smallest |Re lambda| (ties in input order),
    R (n x m) unit right eigenvectors, L (n x m) left eigenvectors with L^H R = I."""
    lam, X = np.linalg.eig(A)
    Xinv = np.linalg.inv(X)
    idx = np.argsort(np.abs(lam.real), kind="stable")[:m]
    return Xinv[idx].conj().T, X[:, idx], lam[idx]


def projector_apply(L, R, b):
    """P b = R (L^H b)."""
    return R @ (L.conj().T @ b)
