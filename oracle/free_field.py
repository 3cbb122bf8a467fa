"""Exact functions of H_W(mu) on a constant abelian SU(3) background (test infrastructure only).

A constant background U_nu(x) = diag(e^{i phi_nu0}, e^{i phi_nu1}, e^{i phi_nu2}) with
phi_nu0 + phi_nu1 + phi_nu2 = 0 is translation invariant, so the Wilson operator of the section
"The overlap operator at nonzero chemical potential" (the hop convention pinned in
tests/test_oracle_operator.py) is block diagonal on plane waves: for colour c and lattice momentum
p (antiperiodic in time: p_t = 2 pi (n + 1/2) / L_t),

    H_W(mu) (e^{i p.x} e_c u) = e^{i p.x} e_c h(q) u,   h(q) = gamma5 (M(q) + i sum_nu gamma_nu s_nu(q)),
    M(q) = 1 - 2 kappa sum_nu cos q_nu,   s_nu(q) = 2 kappa sin q_nu,
    q_nu = p_nu + phi_nu,c   (q_t also + i mu).

Squaring, h(q)^2 = (M^2 + sum_nu s_nu^2) I (the gamma matrices anticommute with gamma5 and each
other), so h(q) has the eigenvalues +-lambda, lambda = sqrt(M^2 + sum s^2) with Re lambda >= 0,
each twice; for an odd scalar function f (sign, or the rational g_s(c t) of Eq. (pfe_s)),
f(h) = (f(lambda) / lambda) h.  With the discrete Fourier transform this gives sign(H_W) b, the
rational approximation, and the LR-deflated form x_P + g_s(cH)(I - P) b of the section
"Deflation" exactly, at any lattice size, in O(V log V).

The critical eigenpairs (the blocks of smallest |Re lambda|; a block holds +-lambda, twice each)
are plane waves times the eigenvectors of the 4 x 4 block, with L^H R = I.
"""
from __future__ import annotations

import numpy as np

from .wilson import gammas


def phases_of(U) -> np.ndarray:
    """(4, 3) phases phi_nu,c of a constant diagonal SU(3) field (canonical link layout);
    raises ValueError for any other field."""
    U = np.asarray(U)
    u0 = U.reshape(-1, 4, 3, 3)[0]
    if not np.allclose(U.reshape(-1, 4, 3, 3), u0[None], rtol=0, atol=1e-14):
        raise ValueError("background is not constant")
    if np.abs(u0 - np.einsum("nii->ni", u0)[:, :, None] * np.eye(3)).max() > 1e-14:
        raise ValueError("background links are not diagonal")
    d = np.einsum("nii->ni", u0)
    if np.abs(np.abs(d) - 1).max() > 1e-14:
        raise ValueError("diagonal entries are not phases")
    return np.angle(d)


class ConstantBackground:
    """sign(H_W(mu)) and friends on a constant diagonal SU(3) field (dims = (Lx, Ly, Lz, Lt),
    periodic space, antiperiodic time)."""

    def __init__(self, U, dims, kappa: float = 0.2):
        self.dims = tuple(int(d) for d in dims)
        self.kappa = float(kappa)
        self.phi = phases_of(U)
        Lx, Ly, Lz, Lt = self.dims
        self.V = Lx * Ly * Lz * Lt
        self.shape = (Lt, Lz, Ly, Lx)
        # lattice momenta on the canonical site grid (t, z, y, x)
        self.p = [2 * np.pi * np.arange(Lx) / Lx, 2 * np.pi * np.arange(Ly) / Ly,
                  2 * np.pi * np.arange(Lz) / Lz, 2 * np.pi * (np.arange(Lt) + 0.5) / Lt]

    # -------------------------------------------------------------- the 4 x 4 blocks
    def _q(self, c: int, mu: float):
        q = [self.p[nu] + self.phi[nu, c] for nu in range(4)]
        q[3] = q[3] + 1j * mu
        return q

    def _grid(self, f, c, mu):
        """f(q_nu) on the (t, z, y, x) momentum grid for nu = x, y, z, t."""
        qx, qy, qz, qt = self._q(c, mu)
        return [f(qx)[None, None, None, :], f(qy)[None, None, :, None], f(qz)[None, :, None, None],
                f(qt)[:, None, None, None]]

    def symbol_parts(self, mu: float):
        """M and s_nu: arrays of shape (Lt, Lz, Ly, Lx, 3) and (4, Lt, Lz, Ly, Lx, 3)."""
        M = np.empty(self.shape + (3,), dtype=np.complex128)
        s = np.empty((4,) + self.shape + (3,), dtype=np.complex128)
        for c in range(3):
            cs = self._grid(np.cos, c, mu)
            sn = self._grid(np.sin, c, mu)
            M[..., c] = 1 - 2 * self.kappa * (cs[0] + cs[1] + cs[2] + cs[3])
            for nu in range(4):
                s[nu, ..., c] = np.broadcast_to(2 * self.kappa * sn[nu], self.shape)
        return M, s

    def block(self, mu: float, t: int, z: int, y: int, x: int, c: int) -> np.ndarray:
        """The 4 x 4 matrix h(q) of one momentum and colour."""
        G = gammas()
        q = [self.p[0][x], self.p[1][y], self.p[2][z], self.p[3][t]]
        q = np.array([q[nu] + self.phi[nu, c] for nu in range(4)], dtype=np.complex128)
        q[3] += 1j * mu
        M = 1 - 2 * self.kappa * np.cos(q).sum()
        s = 2 * self.kappa * np.sin(q)
        return G[4] @ (M * np.eye(4) + 1j * sum(G[nu] * s[nu] for nu in range(4)))

    def lam(self, mu: float) -> np.ndarray:
        """lambda (Re >= 0) of every block, shape (Lt, Lz, Ly, Lx, 3)."""
        M, s = self.symbol_parts(mu)
        l = np.sqrt(M * M + (s * s).sum(axis=0))
        return np.where(l.real < 0, -l, l)

    def _apply_h(self, M, s, bt):
        """h u for every block: bt of shape (Lt, Lz, Ly, Lx, 4, 3) (spin, colour)."""
        G = gammas()
        out = np.einsum("...c,...ac->...ac", M, bt)
        for nu in range(4):
            out = out + 1j * np.einsum("ab,...c,...bc->...ac", G[nu], s[nu], bt)
        return np.einsum("ab,...bc->...ac", G[4], out)

    # -------------------------------------------------------------- Fourier transform
    def fourier(self, b) -> np.ndarray:
        """b~(p) = sum_x e^{-i p.x} b(x) (antiperiodic time through the e^{-i pi t / Lt} twist)."""
        Lt = self.dims[3]
        a = np.asarray(b, dtype=np.complex128).reshape(self.shape + (4, 3))
        tw = np.exp(-1j * np.pi * np.arange(Lt) / Lt)[:, None, None, None, None, None]
        return np.fft.fftn(a * tw, axes=(0, 1, 2, 3))

    def inverse_fourier(self, bt) -> np.ndarray:
        Lt = self.dims[3]
        tw = np.exp(1j * np.pi * np.arange(Lt) / Lt)[:, None, None, None, None, None]
        return np.fft.ifftn(bt, axes=(0, 1, 2, 3)) * tw

    # -------------------------------------------------------------- functions of H
    def apply_odd(self, b, mu: float, f, exact_blocks=None) -> np.ndarray:
        """f(H_W(mu)) b for an odd scalar f (vectorised over a complex array), block by block as
        (f(lambda) / lambda) h; on the blocks flagged in exact_blocks (bool, shape
        (Lt, Lz, Ly, Lx, 3)) sign replaces f: the LR-deflated x_P + f(H)(I - P) b when those
        blocks are the deflated eigenvectors."""
        M, s = self.symbol_parts(mu)
        l = np.sqrt(M * M + (s * s).sum(axis=0))
        l = np.where(l.real < 0, -l, l)
        if np.any(np.abs(l.real) <= 1e-12 * np.abs(l).max()):
            raise ValueError("an eigenvalue lies on the imaginary axis: sign undefined")
        scale = f(l) / l
        if exact_blocks is not None:
            scale = np.where(exact_blocks, 1.0 / l, scale)  # sign(lambda) = 1 for Re lambda > 0
        bt = self.fourier(b)
        out = self._apply_h(M, s, bt) * scale[..., None, :]
        return self.inverse_fourier(out).reshape(np.shape(b))

    def sign(self, b, mu: float) -> np.ndarray:
        """sign(H_W(mu)) b exactly."""
        return self.apply_odd(b, mu, lambda t: np.ones_like(t))

    def rational(self, b, mu: float, omega, sigma, c, exact_blocks=None) -> np.ndarray:
        """g(c H) b with g(t) = t sum_i omega_i / (t^2 - sigma_i), Eq. (pfe_s)."""
        def g(t):
            ct = c * t
            return ct * sum(w / (ct * ct - q) for w, q in zip(omega, sigma))
        return self.apply_odd(b, mu, g, exact_blocks)

    # -------------------------------------------------------------- critical eigenpairs
    def critical_blocks(self, mu: float, nblocks: int):
        """Flat indices (into (Lt, Lz, Ly, Lx, 3)) of the nblocks blocks of smallest |Re lambda|
        and the boolean mask of them; raises ValueError when the cut falls inside a tie."""
        l = self.lam(mu).ravel()
        o = np.argsort(np.abs(l.real), kind="stable")
        if nblocks < l.size and abs(abs(l[o[nblocks]].real) - abs(l[o[nblocks - 1]].real)) <= 1e-12:
            raise ValueError("the cut falls inside a degenerate set")
        mask = np.zeros(l.size, dtype=bool)
        mask[o[:nblocks]] = True
        return o[:nblocks], mask.reshape(self.shape + (3,))

    def deflation_set(self, mu: float, nblocks: int):
        """(lam (4 nblocks,), L, R (4 nblocks, 12 V) canonical vectors): the right eigenvectors
        R_j = e^{i p.x} e_c u_j / sqrt(V) of the critical blocks (u_j the unit eigenvectors of
        the 4 x 4 block) and the left ones with L^H R = I."""
        idx, _ = self.critical_blocks(mu, nblocks)
        Lt, Lz, Ly, Lx = self.shape
        t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
        lams, Ls, Rs = [], [], []
        for f in idx:
            it, iz, iy, ix, c = np.unravel_index(f, self.shape + (3,))
            ph = np.exp(1j * (self.p[0][ix] * x + self.p[1][iy] * y + self.p[2][iz] * z + self.p[3][it] * t))
            ph = ph / np.sqrt(self.V)
            h = self.block(mu, it, iz, iy, ix, c)
            ev, X = np.linalg.eig(h)
            X = X / np.linalg.norm(X, axis=0)
            Y = np.linalg.inv(X)   # rows: left eigenvectors (conjugated), Y X = I
            for j in range(4):
                r = np.zeros(self.shape + (4, 3), dtype=np.complex128)
                l_ = np.zeros_like(r)
                r[..., :, c] = ph[..., None] * X[:, j]
                l_[..., :, c] = ph[..., None] * Y[j, :].conj()
                lams.append(ev[j])
                Rs.append(r.ravel())
                Ls.append(l_.ravel())
        return np.array(lams), np.stack(Ls), np.stack(Rs)
