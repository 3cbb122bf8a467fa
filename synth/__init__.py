"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *generates data*: SU(3) gauge links, source vectors and the
per-problem parameters of batched runs.  It holds none of the arithmetic of
the sign-function method, so the GPU path and the CPU oracle can both consume
its outputs without sharing any code of the method itself.

Canonical layouts (numpy, complex128):
  links  : shape (Lt, Lz, Ly, Lx, 4, 3, 3)  -- U_nu(x), nu = x,y,z,t; row-major
  spinor : shape (Lt, Lz, Ly, Lx, 4, 3)     -- spin index, then colour index
so that the flat site index is x + Lx*(y + Ly*(z + Lz*t)).

Link recipe: U = exp(i*eps*X) with X = sum_a x_a lambda_a / 2, x_a ~ N(0,1)
(traceless Hermitian, Gell-Mann basis), evaluated through the eigenbasis of X.
The paper's quenched beta=5.1 ensembles (numerical-results section) are not
available; these smooth random fields stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "gauge_field",
    "unit_gauge_field",
    "constant_gauge_field",
    "gaussian_source",
    "ones_source",
    "mixed_batch_recipe",
    "lattice_dims",
]


def lattice_dims(spec) -> tuple:
    """Normalise a lattice spec to (Lx, Ly, Lz, Lt).

    Accepts an int L (L^4) or a 4-sequence (Lx, Ly, Lz, Lt)."""
    if isinstance(spec, (int, np.integer)):
        return (int(spec),) * 4
    d = tuple(int(v) for v in spec)
    if len(d) != 4:
        raise ValueError("lattice needs 4 extents (Lx, Ly, Lz, Lt)")
    return d


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _spawn(seed):
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    links_ss, b_ss = ss.spawn(2)
    return links_ss, b_ss


def gauge_field(dims, eps: float, seed=0, chunk: int = 1 << 18) -> np.ndarray:
    """SU(3) links U = exp(i eps X), X Gaussian traceless Hermitian.

    `seed` is an int or a numpy SeedSequence; the links use the first child of
    seed.spawn(2), the source vector the second (see gaussian_source)."""
    Lx, Ly, Lz, Lt = lattice_dims(dims)
    links_ss, _ = _spawn(seed)
    rng = np.random.default_rng(links_ss)
    xs = rng.standard_normal((Lt, Lz, Ly, Lx, 4, 8))
    lam = gell_mann()
    flat = xs.reshape(-1, 8)
    out = np.empty((flat.shape[0], 3, 3), dtype=np.complex128)
    for s in range(0, flat.shape[0], chunk):
        X = np.einsum("na,aij->nij", flat[s:s + chunk], lam) * 0.5
        w, V = np.linalg.eigh(X)
        ph = np.exp(1j * eps * w)
        out[s:s + chunk] = np.einsum("nij,nj,nkj->nik", V, ph, V.conj())
    return out.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)


def unit_gauge_field(dims) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    Lx, Ly, Lz, Lt = lattice_dims(dims)
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def constant_gauge_field(dims, seed=0) -> np.ndarray:
    """Constant diagonal SU(3) links U_nu = diag(e^{i a}, e^{i b}, e^{-i (a + b)}), the phases
    a, b of each direction uniform in [-pi, pi) from the seed: a translation-invariant background
    whose colours see different momenta."""
    Lx, Ly, Lz, Lt = lattice_dims(dims)
    ph = np.random.default_rng(np.random.SeedSequence([seed, 7])).uniform(-np.pi, np.pi, (4, 2))
    d = np.exp(1j * np.concatenate([ph, -ph.sum(axis=1, keepdims=True)], axis=1))
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    for c in range(3):
        U[..., c, c] = d[:, c]
    return U


def gaussian_source(dims, seed=0) -> np.ndarray:
    """Complex Gaussian source vector, normalised to unit 2-norm."""
    Lx, Ly, Lz, Lt = lattice_dims(dims)
    _, b_ss = _spawn(seed)
    g = np.random.default_rng(b_ss).standard_normal((2, Lt, Lz, Ly, Lx, 4, 3))
    b = g[0] + 1j * g[1]
    return b / np.linalg.norm(b)


def ones_source(dims) -> np.ndarray:
    """The source b = (1, ..., 1) of the paper's numerical section, normalised."""
    Lx, Ly, Lz, Lt = lattice_dims(dims)
    b = np.ones((Lt, Lz, Ly, Lx, 4, 3), dtype=np.complex128)
    return b / np.linalg.norm(b)


def mixed_batch_recipe(nrhs: int = 32, sizes=(8, 12, 16), eps: float = 0.4,
                       mu_max: float = 0.3, seed: int = 0):
    """Problem list for a batch of right-hand sides spread over uneven lattices.

    One gauge field per lattice size (seeds from SeedSequence(seed).spawn(len(sizes))),
    right-hand side j lives on size j mod len(sizes), with its own chemical
    potential mu_j ~ U[0, mu_max] and its own Gaussian source.  Returns
    (fields, problems) where fields[i] = (dims, U) and problems[j] =
    (field_index, mu_j, b_j)."""
    root = np.random.SeedSequence(seed)
    fseeds = root.spawn(len(sizes))
    fields = [(lattice_dims(L), gauge_field(L, eps, fs)) for L, fs in zip(sizes, fseeds)]
    prng = np.random.default_rng(np.random.SeedSequence([seed, 1]))
    problems = []
    for j in range(nrhs):
        fi = j % len(sizes)
        mu = float(prng.uniform(0.0, mu_max))
        bseed = np.random.SeedSequence([seed, 2, j])
        problems.append((fi, mu, gaussian_source(fields[fi][0], bseed)))
    return fields, problems
