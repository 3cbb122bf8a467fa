"""Pins of the oracle's exact functions of H_W on a constant SU(3) background.

The closed form (plane waves, 4 x 4 blocks with h^2 = lambda^2 I) is checked against
independent routes: the naive per-site operator applied to plane waves and to random
vectors, the dense matrix sign and the dense rational function on tiny lattices, and the
eigen-relations of the deflation set with the naive operator and its independently written
adjoint.  A sign slip in a momentum, a dropped twist of the antiperiodic time direction, a
wrong branch of lambda or a transposed left eigenvector each fails one of them.
"""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, rational
from oracle.dense import rational_dense, sign_eig
from oracle.free_field import ConstantBackground, phases_of

from conftest import rel


def test_phases_of_rejects_other_fields():
    dims = (2, 2, 2, 4)
    with pytest.raises(ValueError):
        phases_of(synth.gauge_field(dims, 0.4, 0))
    U = synth.constant_gauge_field(dims, 3)
    ph = phases_of(U)
    assert np.allclose(np.exp(1j * ph.sum(axis=1)), 1, atol=1e-14)


@pytest.mark.parametrize("mu", [0.0, 0.3, -0.2])
def test_blocks_match_naive_operator_on_plane_waves(mu, rng):
    dims = (4, 6, 4, 8)
    U = synth.constant_gauge_field(dims, 1)
    W = WilsonRef(U, dims, 0.2)
    F = ConstantBackground(U, dims, 0.2)
    Lt, Lz, Ly, Lx = F.shape
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    for (it, iz, iy, ix, c) in [(0, 0, 0, 0, 0), (3, 1, 5, 2, 1), (7, 3, 2, 1, 2)]:
        ph = np.exp(1j * (F.p[0][ix] * x + F.p[1][iy] * y + F.p[2][iz] * z + F.p[3][it] * t))
        u = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        psi = np.zeros(F.shape + (4, 3), dtype=np.complex128)
        psi[..., :, c] = ph[..., None] * u
        want = np.zeros_like(psi)
        want[..., :, c] = ph[..., None] * (F.block(mu, it, iz, iy, ix, c) @ u)
        assert np.abs(W.apply(psi, mu) - want).max() < 1e-13


@pytest.mark.parametrize("mu", [0.0, 0.25])
def test_odd_identity_function_is_the_operator(mu, rng):
    """f(t) = t through the Fourier route equals the naive operator on a random vector."""
    dims = (6, 4, 4, 8)
    U = synth.constant_gauge_field(dims, 2)
    b = synth.gaussian_source(dims, 5)
    got = ConstantBackground(U, dims, 0.2).apply_odd(b, mu, lambda t: t)
    assert rel(got, WilsonRef(U, dims, 0.2).apply(b, mu)) < 1e-13


def test_block_square_is_scalar():
    dims = (4, 4, 4, 6)
    F = ConstantBackground(synth.constant_gauge_field(dims, 4), dims, 0.2)
    lam = F.lam(0.3)
    for (it, iz, iy, ix, c) in [(0, 0, 0, 0, 0), (5, 2, 1, 3, 2), (2, 3, 3, 0, 1)]:
        h = F.block(0.3, it, iz, iy, ix, c)
        l = lam[it, iz, iy, ix, c]
        assert np.abs(h @ h - l * l * np.eye(4)).max() < 1e-13
        assert l.real >= 0
        assert np.allclose(np.sort_complex(np.linalg.eigvals(h)), np.sort_complex(np.array([l, l, -l, -l])),
                           atol=1e-7)


@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("dims,seed", [((2, 2, 2, 4), 0), ((2, 2, 4, 4), 6)])
def test_sign_and_rational_match_dense(mu, dims, seed):
    U = synth.constant_gauge_field(dims, seed)
    b = synth.gaussian_source(dims, seed).ravel()
    A = WilsonRef(U, dims, 0.2).dense(mu)
    F = ConstantBackground(U, dims, 0.2)
    assert rel(F.sign(b, mu), sign_eig(A, b)) < 1e-10
    om, sg, c = rational.coefficients(12, 0.15, 2.7)
    assert rel(F.rational(b, mu, om, sg, c), rational_dense(A, b, om, sg, c)) < 1e-12


def test_sign_squares_to_identity():
    dims = (4, 4, 6, 8)
    U = synth.constant_gauge_field(dims, 8)
    F = ConstantBackground(U, dims, 0.2)
    b = synth.gaussian_source(dims, 1)
    sb = F.sign(b, 0.2)
    assert rel(F.sign(sb, 0.2), b) < 1e-13
    W = WilsonRef(U, dims, 0.2)
    assert rel(F.sign(W.apply(b, 0.2), 0.2), W.apply(sb, 0.2)) < 1e-13


def test_deflation_set_eigen_relations():
    dims = (4, 4, 4, 6)
    U = synth.constant_gauge_field(dims, 3)
    mu = 0.2
    F = ConstantBackground(U, dims, 0.2)
    lam, L, R = F.deflation_set(mu, 3)
    assert lam.shape == (12,) and L.shape == R.shape == (12, 12 * F.V)
    W = WilsonRef(U, dims, 0.2)
    for j in range(12):
        assert np.linalg.norm(W.apply(R[j], mu) - lam[j] * R[j]) < 1e-13 * abs(lam[j])
        assert np.linalg.norm(W.apply_adj(L[j], mu) - np.conj(lam[j]) * L[j]) < 1e-12 * np.linalg.norm(L[j]) * abs(lam[j])
        assert abs(np.linalg.norm(R[j]) - 1) < 1e-13
    assert np.abs(L.conj() @ R.T - np.eye(12)).max() < 1e-12


def test_critical_blocks_are_the_smallest_of_the_dense_spectrum():
    dims = (2, 2, 4, 4)
    U = synth.constant_gauge_field(dims, 6)
    mu = 0.25
    F = ConstantBackground(U, dims, 0.2)
    lam, L, R = F.deflation_set(mu, 2)
    ev = np.linalg.eigvals(WilsonRef(U, dims, 0.2).dense(mu))
    dense_re = np.sort(np.abs(ev.real))
    assert np.allclose(np.sort(np.abs(lam.real)), dense_re[:8], atol=1e-7)
    assert dense_re[8] > dense_re[7] + 1e-6   # the cut lies in a gap


def test_deflated_rational_matches_dense_projection():
    """x_P + g(cH)(I - P) b (Eq. exact_proj with the dense matrices) equals the block form with
    sign on the deflated blocks."""
    dims = (2, 2, 4, 4)
    U = synth.constant_gauge_field(dims, 6)
    mu = 0.25
    b = synth.gaussian_source(dims, 2).ravel()
    F = ConstantBackground(U, dims, 0.2)
    lam, L, R = F.deflation_set(mu, 2)
    _, mask = F.critical_blocks(mu, 2)
    A = WilsonRef(U, dims, 0.2).dense(mu)
    om, sg, c = rational.coefficients(10, 0.2, 2.7)
    xP = R.T @ (np.sign(lam.real) * (L.conj() @ b))
    bP = b - R.T @ (L.conj() @ b)
    want = xP + rational_dense(A, bP, om, sg, c)
    assert rel(F.rational(b, mu, om, sg, c, exact_blocks=mask), want) < 1e-12
