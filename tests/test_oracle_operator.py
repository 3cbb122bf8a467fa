"""Pins of the oracle's Wilson operator against facts fixed by the mathematics.

The paper defers the definition of D_W(mu) to its reference on the overlap
operator at nonzero chemical potential; the reading pinned here is the one
stated in oracle/wilson_ref.c.  Each test targets a different class of
mistake: the free-field plane waves fix every hop sign, projector orientation,
the e^{-+mu} weights and the boundary factors; gamma5-hermiticity ties the
independently written adjoint to the forward operator; gauge covariance fixes
which link (and which adjoint) each hop uses.
"""
import numpy as np
import pytest

import synth
from oracle import WilsonRef
from oracle.wilson import gammas

from conftest import rel


def _plane_wave(dims, nvec, u):
    Lx, Ly, Lz, Lt = dims
    p = np.array([2 * np.pi * nvec[0] / Lx, 2 * np.pi * nvec[1] / Ly,
                  2 * np.pi * nvec[2] / Lz, 2 * np.pi * (nvec[3] + 0.5) / Lt])
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return p, ph[..., None, None] * u, ph


def _free_symbol(p, kappa, mu):
    """D(p) = M + i sum_nu gamma_nu s_nu, M = 1 - 2 kappa sum cos q, s = 2 kappa sin q,
    q = (p1, p2, p3, p4 + i mu): Fourier transform of the free Wilson operator."""
    G = gammas()
    q = p.astype(np.complex128)
    q[3] += 1j * mu
    M = 1 - 2 * kappa * np.cos(q).sum()
    s = 2 * kappa * np.sin(q)
    return M * np.eye(4) + 1j * sum(G[i] * s[i] for i in range(4))


def test_gamma_matrices_clifford():
    G = gammas()
    for a in range(4):
        assert np.allclose(G[a], G[a].conj().T, atol=1e-15)
        for b in range(4):
            ac = G[a] @ G[b] + G[b] @ G[a]
            assert np.allclose(ac, 2 * np.eye(4) * (a == b), atol=1e-15)
    assert np.allclose(G[4], np.diag([1, 1, -1, -1]), atol=1e-15)


@pytest.mark.parametrize("eps,seed", [(0.5, 0), (0.4, 3)])
def test_links_are_su3(eps, seed):
    U = synth.gauge_field((4, 4, 4, 6), eps, seed).reshape(-1, 3, 3)
    I = np.eye(3)
    assert np.abs(np.einsum("nji,njk->nik", U.conj(), U) - I).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


@pytest.mark.parametrize("mu", [0.0, 0.3, -0.2, 0.7])
@pytest.mark.parametrize("dims,nvec", [((4, 6, 8, 10), (1, 2, 3, 4)),
                                       ((3, 5, 4, 6), (2, 0, 1, 5)),
                                       ((4, 4, 4, 4), (0, 0, 0, 0))])
def test_free_field_plane_waves(dims, nvec, mu, rng):
    kappa = 0.2
    W = WilsonRef(synth.unit_gauge_field(dims), dims, kappa)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p, psi, ph = _plane_wave(dims, nvec, u)
    Dp = _free_symbol(p, kappa, mu)
    got = W.apply(psi, mu, g5=False)
    assert np.abs(got - ph[..., None, None] * (Dp @ u)).max() < 1e-13
    G5 = gammas()[4]
    got5 = W.apply(psi, mu, g5=True)
    assert np.abs(got5 - ph[..., None, None] * (G5 @ Dp @ u)).max() < 1e-13


def test_plane_wave_pin_rejects_wrong_conventions(rng):
    """The closed form separates the stated reading from its look-alikes:
    swapped e^{+-mu} orientation (mu -> -mu), periodic time, wrong kappa."""
    dims, mu, kappa = (4, 4, 4, 6), 0.3, 0.2
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p, psi, ph = _plane_wave(dims, (1, 0, 2, 1), u)
    want = ph[..., None, None] * (_free_symbol(p, kappa, mu) @ u)
    U = synth.unit_gauge_field(dims)
    assert rel(WilsonRef(U, dims, kappa).apply(psi, -mu, g5=False), want) > 1e-3
    assert rel(WilsonRef(U, dims, kappa, bc=(1, 1, 1, 1)).apply(psi, mu, g5=False), want) > 1e-3
    assert rel(WilsonRef(U, dims, 0.19).apply(psi, mu, g5=False), want) > 1e-3


def _match_multisets(a, b):
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(a[:, None] - b[None, :])
    i, j = linear_sum_assignment(cost)
    return cost[i, j].max()


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_free_field_dense_spectrum(mu):
    """Eigenvalues of H_W are +-sqrt(M(q)^2 + sum s_nu(q)^2), each 6-fold."""
    dims, kappa = (2, 2, 2, 4), 0.2
    W = WilsonRef(synth.unit_gauge_field(dims), dims, kappa)
    ev = np.linalg.eigvals(W.dense(mu))
    Lx, Ly, Lz, Lt = dims
    cf = []
    for a in range(Lx):
        for b in range(Ly):
            for c in range(Lz):
                for d in range(Lt):
                    q = np.array([2 * np.pi * a / Lx, 2 * np.pi * b / Ly, 2 * np.pi * c / Lz,
                                  2 * np.pi * (d + 0.5) / Lt], dtype=np.complex128)
                    q[3] += 1j * mu
                    lam = np.sqrt((1 - 2 * kappa * np.cos(q).sum()) ** 2 + ((2 * kappa * np.sin(q)) ** 2).sum())
                    cf += [lam] * 6 + [-lam] * 6
    assert _match_multisets(ev, np.array(cf)) < 1e-6   # degenerate eigenvalues: sqrt(eps) sensitivity


@pytest.mark.parametrize("mu", [0.0, 0.3, -0.25])
def test_gamma5_hermiticity(mu):
    """H_W(mu)^H = H_W(-mu): the independent adjoint against the forward operator."""
    dims = (4, 4, 6, 4)
    W = WilsonRef(synth.gauge_field(dims, 0.5, 7), dims, 0.2)
    phi = synth.gaussian_source(dims, 11)
    psi = synth.gaussian_source(dims, 12)
    assert rel(W.apply_adj(phi, mu), W.apply(phi, -mu)) < 1e-14
    assert abs(np.vdot(phi, W.apply(psi, mu)) - np.vdot(W.apply_adj(phi, mu), psi)) < 1e-14
    # D_W(mu)^H = gamma5 D_W(-mu) gamma5 on the un-multiplied operator
    G5 = gammas()[4]
    lhs = W.apply_adj(phi, mu, g5=False)
    rhs = np.einsum("st,...tc->...sc", G5, W.apply(np.einsum("st,...tc->...sc", G5, phi), -mu, g5=False))
    assert rel(lhs, rhs) < 1e-14


def test_hermitian_at_zero_mu():
    dims = (2, 2, 2, 4)
    W = WilsonRef(synth.gauge_field(dims, 0.5, 1), dims, 0.2)
    H = W.dense(0.0)
    assert np.abs(H - H.conj().T).max() < 1e-15
    H3 = W.dense(0.3)
    assert np.abs(H3 - H3.conj().T).max() > 1e-2


def test_gauge_covariance():
    """U_nu(x) -> G(x) U_nu(x) G(x+nu)^H, psi -> G psi  gives  H -> G H G^H."""
    dims = (4, 4, 4, 6)
    Lx, Ly, Lz, Lt = dims
    U = synth.gauge_field(dims, 0.5, 2)
    Gf = synth.gauge_field(dims, 2.0, 9)[..., 0, :, :]            # one SU(3) matrix per site
    shifts = [(3, 1), (2, 1), (1, 1), (0, 1)]                      # axis of x, y, z, t in (t,z,y,x)
    UG = np.empty_like(U)
    for nu, (ax, _) in enumerate(shifts):
        Gp = np.roll(Gf, -1, axis=ax)                              # G(x + nu)
        UG[..., nu, :, :] = Gf @ U[..., nu, :, :] @ np.conj(np.swapaxes(Gp, -1, -2))
    psi = synth.gaussian_source(dims, 4)
    for mu in (0.0, 0.3):
        a = WilsonRef(UG, dims, 0.2).apply(np.einsum("...ab,...sb->...sa", Gf, psi), mu)
        b = np.einsum("...ab,...sb->...sa", Gf, WilsonRef(U, dims, 0.2).apply(psi, mu))
        assert rel(a, b) < 1e-14


def test_mu_as_twisted_boundary():
    """E^{-1} D_W(mu) E with E = diag(e^{mu t}) is D_W(0) with time-wrap factors
    -e^{-mu Lt} (forward) and -e^{+mu Lt} (backward): equal spectra."""
    dims, mu = (2, 2, 2, 4), 0.3
    U = synth.gauge_field(dims, 0.5, 5)
    Lt = dims[3]
    ev1 = np.linalg.eigvals(WilsonRef(U, dims, 0.2).dense(mu))
    tw = WilsonRef(U, dims, 0.2, bc_fwd=(1, 1, 1, -np.exp(-mu * Lt)), bc_bwd=(1, 1, 1, -np.exp(mu * Lt)))
    ev2 = np.linalg.eigvals(tw.dense(0.0))
    assert _match_multisets(ev1, ev2) < 1e-10


def test_sampled_sites_match_full_apply():
    dims = (4, 6, 4, 8)
    W = WilsonRef(synth.gauge_field(dims, 0.4, 0), dims, 0.2)
    psi = synth.gaussian_source(dims, 0)
    full = W.apply(psi, 0.2).reshape(-1, 4, 3)
    sites = np.array([0, 5, 97, 500, W.V - 1])
    assert np.abs(W.apply_sites(psi, 0.2, sites) - full[sites]).max() == 0.0
