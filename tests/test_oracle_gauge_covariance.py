"""The premise of the library's temporal-gauge lattices, checked on the oracle (CPU only): a
site-local colour rotation G(x) in SU(3) maps the Wilson operator to G H_W G^H when the links
become G(x) U_nu(x) G(x+nu)^H, and the choice G(x, 0) = 1, G(x, t+1) = G(x, t) U_t(x, t) leaves
unit time links everywhere but on the last slice.  sign then commutes with the rotation."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, dense

DIMS = (2, 2, 2, 4)


def _temporal_gauge(U, dims):
    """G per site and the rotated links, canonical layout (site index x fastest)."""
    L0, L1, L2, L3 = dims
    Uc = U.reshape(-1, 4, 3, 3)
    V, vs = Uc.shape[0], L0 * L1 * L2
    G = np.zeros((V, 3, 3), complex)
    for x in range(vs):
        g = np.eye(3, dtype=complex)
        for t in range(L3):
            G[t * vs + x] = g
            g = g @ Uc[t * vs + x, 3]
    stride = (1, L0, L0 * L1, vs)
    Up = np.empty_like(Uc)
    for s in range(V):
        c = (s % L0, (s // L0) % L1, (s // (L0 * L1)) % L2, s // vs)
        for nu in range(4):
            n = s - (dims[nu] - 1) * stride[nu] if c[nu] == dims[nu] - 1 else s + stride[nu]
            Up[s, nu] = G[s] @ Uc[s, nu] @ G[n].conj().T
    return G, Up.reshape(U.shape)


def _rotation(G):
    """the n x n matrix acting as G(x) on the colour index of every spin at every site"""
    V = G.shape[0]
    R = np.zeros((12 * V, 12 * V), complex)
    for s in range(V):
        for sp in range(4):
            i = 12 * s + 3 * sp
            R[i:i + 3, i:i + 3] = G[s]
    return R


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_rotated_operator_and_sign(mu):
    U = synth.gauge_field(DIMS, 0.5, 0)
    G, Up = _temporal_gauge(U, DIMS)
    vs = DIMS[0] * DIMS[1] * DIMS[2]
    Uc = Up.reshape(-1, 4, 3, 3)
    # unit time links off the last slice; unitary rotations
    assert np.abs(Uc[: (DIMS[3] - 1) * vs, 3] - np.eye(3)).max() < 1e-13
    assert np.abs(np.einsum("sij,skj->sik", G, G.conj()) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(G) - 1).max() < 1e-13
    R = _rotation(G)
    H = WilsonRef(U, DIMS, 0.2).dense(mu)
    Hp = WilsonRef(Up, DIMS, 0.2).dense(mu)
    assert np.abs(Hp - R @ H @ R.conj().T).max() < 1e-13
    b = synth.gaussian_source(DIMS, 1).ravel()
    x = dense.sign_schur(H, b)
    xp = R.conj().T @ dense.sign_schur(Hp, R @ b)
    assert np.linalg.norm(xp - x) / np.linalg.norm(x) < 1e-11


def test_a_plain_relabelling_is_not_enough():
    """A planted mistake fails: rotating the links but not the source (or the result) does not give
    sign(H) b, so the library must rotate both sides."""
    U = synth.gauge_field(DIMS, 0.5, 0)
    G, Up = _temporal_gauge(U, DIMS)
    H = WilsonRef(U, DIMS, 0.2).dense(0.3)
    Hp = WilsonRef(Up, DIMS, 0.2).dense(0.3)
    b = synth.gaussian_source(DIMS, 1).ravel()
    x = dense.sign_schur(H, b)
    assert np.linalg.norm(dense.sign_schur(Hp, b) - x) / np.linalg.norm(x) > 1e-2
