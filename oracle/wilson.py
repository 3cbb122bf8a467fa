"""ctypes front end of the oracle's C reference operator (test infrastructure only).

H_W(mu) = gamma5 D_W(mu) with the reading of D_W stated in wilson_ref.c.  The
adjoint comes from an independent routine (conjugate transposes of the hop
blocks), never from the mu -> -mu identity.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_wilson.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
    i64p = C.POINTER(C.c_int64)
    lib.oracle_dirac.argtypes = [dp, dp, dp, ip, C.c_double, C.c_double, dp, dp, C.c_int]
    lib.oracle_dirac_adj.argtypes = [dp, dp, dp, ip, C.c_double, C.c_double, dp, dp, C.c_int, dp]
    lib.oracle_dirac_sites.argtypes = [dp, dp, dp, ip, C.c_double, C.c_double, dp, dp, C.c_int,
                                       i64p, C.c_int64]
    lib.oracle_gammas.argtypes = [dp]
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_get_threads.restype = C.c_int
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def gammas() -> np.ndarray:
    """(5, 4, 4): gamma_1..gamma_4 and gamma5 = gamma1 gamma2 gamma3 gamma4 as used by the oracle."""
    out = np.zeros((5, 4, 4), dtype=np.complex128)
    _load().oracle_gammas(_dp(out))
    return out


class WilsonRef:
    """H_W(mu) = gamma5 D_W(mu) on one gauge field, FP64, CPU.

    dims = (Lx, Ly, Lz, Lt); links in canonical layout (Lt,Lz,Ly,Lx,4,3,3);
    bc = boundary factor per direction for hops that wrap (periodic space,
    antiperiodic time by default).  `bc_fwd`/`bc_bwd` allow distinct complex
    factors for forward and backward wrapping hops (twisted boundaries)."""

    def __init__(self, U, dims, kappa: float = 0.2, bc=(1, 1, 1, -1), bc_fwd=None, bc_bwd=None):
        self.dims = tuple(int(d) for d in dims)
        Lx, Ly, Lz, Lt = self.dims
        self.U = np.ascontiguousarray(U, dtype=np.complex128).reshape(Lt, Lz, Ly, Lx, 4, 3, 3)
        self.kappa = float(kappa)
        self.V = Lx * Ly * Lz * Lt
        self.n = 12 * self.V
        bf = np.asarray(bc if bc_fwd is None else bc_fwd, dtype=np.complex128)
        bb = np.asarray(bc if bc_bwd is None else bc_bwd, dtype=np.complex128)
        self._bf = np.ascontiguousarray(bf)
        self._bb = np.ascontiguousarray(bb)
        self._L = (C.c_int * 4)(*self.dims)
        self.shape = (Lt, Lz, Ly, Lx, 4, 3)

    def _vec(self, psi):
        a = np.ascontiguousarray(psi, dtype=np.complex128)
        if a.size != self.n:
            raise ValueError(f"spinor has {a.size} entries, lattice needs {self.n}")
        return a

    def apply(self, psi, mu: float, g5: bool = True) -> np.ndarray:
        """gamma5 D_W(mu) psi (g5=False: D_W(mu) psi)."""
        a = self._vec(psi)
        out = np.empty_like(a)
        _load().oracle_dirac(_dp(self.U), _dp(a), _dp(out), self._L, self.kappa, float(mu),
                             _dp(self._bf), _dp(self._bb), int(bool(g5)))
        return out.reshape(np.shape(psi))

    def apply_adj(self, psi, mu: float, g5: bool = True) -> np.ndarray:
        """(gamma5 D_W(mu))^H psi from the conjugate-transposed hop blocks."""
        a = self._vec(psi)
        out = np.empty_like(a)
        scratch = np.empty_like(a)
        _load().oracle_dirac_adj(_dp(self.U), _dp(a), _dp(out), self._L, self.kappa, float(mu),
                                 _dp(self._bf), _dp(self._bb), int(bool(g5)), _dp(scratch))
        return out.reshape(np.shape(psi))

    def apply_sites(self, psi, mu: float, sites, g5: bool = True) -> np.ndarray:
        """Rows of gamma5 D_W(mu) psi at the given flat site indices, shape (len(sites), 4, 3)."""
        a = self._vec(psi)
        s = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty((s.size, 4, 3), dtype=np.complex128)
        _load().oracle_dirac_sites(_dp(self.U), _dp(a), _dp(out), self._L, self.kappa, float(mu),
                                   _dp(self._bf), _dp(self._bb), int(bool(g5)),
                                   s.ctypes.data_as(C.POINTER(C.c_int64)), s.size)
        return out

    def dense(self, mu: float, g5: bool = True) -> np.ndarray:
        """The n x n matrix, assembled column by column from unit vectors (n <= a few 1000)."""
        n = self.n
        if n > 6144:
            raise ValueError("dense assembly is meant for tiny lattices")
        M = np.empty((n, n), dtype=np.complex128)
        e = np.zeros(n, dtype=np.complex128)
        for j in range(n):
            e[j] = 1.0
            M[:, j] = self.apply(e, mu, g5)
            e[j] = 0.0
        return M
