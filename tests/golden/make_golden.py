"""Write the stored expected values under tests/golden/ (calls only oracle/ and synth/).

    python tests/golden/make_golden.py

c1_dense.npz -- the 4^4 configuration (links eps = 0.5, seed 0; kappa = 0.2,
    mu = 0.3; Gaussian source of seed 0):
      sign_b   sign(H_W) b from the eigendecomposition of the dense H_W
               (definition f(A) = R f(Lambda) R^{-1}, sign z = sign Re z;
               introduction, Eqs. (1), (matfun_action))
      g16_b    g_16(cA) b, the 16-pole Neuberger approximation (Eq. (pfe_s))
               with c from the spectral-circle heuristic through the smallest
               and largest eigenvalue moduli (numerical-results section)
      g16_g16_b  g_16(cA) applied to g16_b (same coefficients)
      acc16    the accuracy measure 1/2 ||g_16(cA)^2 b - b|| / ||b|| of the
               numerical-results section for this approximation
      alpha, beta  smallest / largest |lambda| of H_W
      evals    all eigenvalues of H_W
c1_deflation.npz -- the same configuration and source, LR deflation of the m = 15
    eigenvalues closest to the imaginary axis (section "Deflation"; the widest
    relative gap in |Re lambda| among the first 24):
      lam      the 15 critical eigenvalues (ordered by |Re lambda|)
      Pb       P b = R_m L_m^H b
      xP       x_P = R_m sign(Lambda_m) L_m^H b (Eq. (exact_proj))
      alpha_rest  smallest |lambda| of the non-deflated eigenvalues
Dense n = 3072 eigendecompositions: about a minute each on 8 cores.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import WilsonRef, dense, eigen, rational  # noqa: E402


def c1():
    dims, eps, seed, kappa, mu = (4, 4, 4, 4), 0.5, 0, 0.2, 0.3
    U = synth.gauge_field(dims, eps, seed)
    b = synth.gaussian_source(dims, seed).ravel()
    H = WilsonRef(U, dims, kappa).dense(mu)
    evals = np.linalg.eigvals(H)
    alpha, beta = float(np.abs(evals).min()), float(np.abs(evals).max())
    sign_b = dense.sign_eig(H, b)
    om, sg, c = rational.coefficients(16, alpha, beta)
    g16_b = dense.rational_dense(H, b, om, sg, c)
    g16_g16_b = dense.rational_dense(H, g16_b, om, sg, c)
    acc16 = 0.5 * np.linalg.norm(g16_g16_b - b) / np.linalg.norm(b)
    np.savez_compressed(os.path.join(HERE, "c1_dense.npz"), sign_b=sign_b, g16_b=g16_b, alpha=alpha,
                        beta=beta, evals=evals, g16_g16_b=g16_g16_b, acc16=acc16)
    print("c1: alpha", alpha, "beta", beta, "|g16 - sign| / |sign|",
          np.linalg.norm(g16_b - sign_b) / np.linalg.norm(sign_b), "accuracy measure", acc16)


def c1_deflation():
    dims, eps, seed, kappa, mu, m = (4, 4, 4, 4), 0.5, 0, 0.2, 0.3, 15
    U = synth.gauge_field(dims, eps, seed)
    b = synth.gaussian_source(dims, seed).ravel()
    H = WilsonRef(U, dims, kappa).dense(mu)
    L, R, lam = eigen.critical_eigenpairs(H, m)
    c = L.conj().T @ b
    Pb = R @ c
    xP = R @ (np.sign(lam.real) * c)
    evals = np.linalg.eigvals(H)
    rest = evals[np.argsort(np.abs(evals.real))[m:]]
    alpha_rest = float(np.abs(rest).min())
    np.savez_compressed(os.path.join(HERE, "c1_deflation.npz"), lam=lam, Pb=Pb, xP=xP, alpha_rest=alpha_rest)
    print("c1_deflation: |Re lam| of the deflated", np.abs(lam.real).min(), "..", np.abs(lam.real).max(),
          "alpha of the rest", alpha_rest)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c1_deflation"]
    if "c1" in which:
        c1()
    if "c1_deflation" in which:
        c1_deflation()
