"""Host parity of the small-matrix sign (sgn_small_sign) with the oracle's dense routes.

The library routine runs on the CPU (no GPU needed): tridiagonal matrices from the
oracle's two-sided Lanczos on small Wilson operators (mu = 0: Hermitian, real symmetric
T; mu > 0: non-Hermitian, with the near-duplicate eigenvalues that loss of
biorthogonality brings at larger k) and random non-normal tridiagonals, against
sign(T) e_1 by the oracle's eigendecomposition / Schur-Sylvester route."""
import time

import numpy as np
import pytest

import synth
import paper_0910_1048_amd as sgn
from oracle import WilsonRef, krylov

from conftest import rel


def _parts(T):
    k = T.shape[0]
    return np.diag(T).copy(), np.array([T[i + 1, i] for i in range(k - 1)]), \
        np.array([T[i, i + 1] for i in range(k - 1)])


def _lanczos_T(dims, mu, k, seed=0):
    W = WilsonRef(synth.gauge_field(dims, 0.5, seed), dims, 0.2)
    b = synth.gaussian_source(dims, seed).ravel()
    v1 = b / np.linalg.norm(b)
    _, T, _ = krylov.two_sided_lanczos(lambda v: W.apply(v, mu), lambda v: W.apply_adj(v, mu), v1, v1.copy(), k)
    return T


@pytest.mark.parametrize("mu,k", [(0.0, 40), (0.1, 60), (0.2, 300), (0.3, 200)])
def test_lanczos_tridiagonals_match_oracle(mu, k):
    T = _lanczos_T((4, 4, 4, 4), mu, k)
    t0 = time.perf_counter()
    y, mr = sgn.sgn_small_sign(*_parts(T))
    dt = time.perf_counter() - t0
    want = krylov.small_sign_e1(T)
    print(f"mu={mu} k={k}: {dt * 1e3:.2f} ms, rel err {rel(y, want):.1e}")
    assert rel(y, want) < 1e-11
    assert mr == pytest.approx(np.min(np.abs(np.linalg.eigvals(T).real)), rel=1e-8)


def test_random_nonnormal_tridiagonals(rng):
    for k in (2, 3, 10, 50):
        d = np.where(rng.random(k) < 0.5, -1, 1) * rng.uniform(0.5, 2, k) + 0.3j * rng.standard_normal(k)
        lo = 0.3 * (rng.standard_normal(k - 1) + 1j * rng.standard_normal(k - 1))
        up = 0.3 * (rng.standard_normal(k - 1) + 1j * rng.standard_normal(k - 1))
        T = np.diag(d) + np.diag(lo, -1) + np.diag(up, 1)
        y, _ = sgn.sgn_small_sign(d, lo, up)
        assert rel(y, krylov.small_sign_e1(T)) < 1e-11, k


def test_hermitian_case_and_one_by_one():
    T = _lanczos_T((2, 2, 2, 4), 0.0, 30)
    assert np.allclose(T, T.conj().T, atol=1e-12)
    y, _ = sgn.sgn_small_sign(*_parts(T))
    lam, X = np.linalg.eigh(T)
    want = X @ (np.sign(lam) * X[0].conj())
    assert rel(y, want) < 1e-12
    y1, mr = sgn.sgn_small_sign([-0.7 + 0.2j], [], [])
    assert y1[0] == -1.0 and mr == pytest.approx(0.7)


def test_errors():
    with pytest.raises(sgn.SgnError) as e:
        sgn.sgn_small_sign([0.0, 0.0], [-1.0], [1.0])  # eigenvalues +-i
    assert e.value.status == 6  # SGN_ERR_IMAG_AXIS
    with pytest.raises(sgn.SgnError) as e:
        sgn.sgn_small_sign([], [], [])
    assert e.value.status == 1
    with pytest.raises(sgn.SgnError) as e:
        sgn.sgn_small_sign([1.0, np.nan], [0.5], [0.5])
    assert e.value.status == 1


def test_baseline_isa_build_matches_oracle():
    """The Schur routine is built for AVX2/FMA and for baseline x86-64; the library picks one
    per host.  SGN_HOST_ISA=baseline forces the baseline build in a fresh process."""
    import os
    import subprocess
    import sys
    code = (
        "import numpy as np, sys\n"
        "sys.path.insert(0, 'tests')\n"
        "from test_small_sign_host import _lanczos_T, _parts\n"
        "import paper_0910_1048_amd as sgn\n"
        "from oracle import krylov\n"
        "T = _lanczos_T((4, 4, 4, 4), 0.3, 200)\n"
        "y, _ = sgn.sgn_small_sign(*_parts(T))\n"
        "w = krylov.small_sign_e1(T)\n"
        "print(np.linalg.norm(y - w) / np.linalg.norm(w))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, SGN_HOST_ISA="baseline")
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    err = float(out.stdout.strip().splitlines()[-1])
    print(f"baseline build: rel err {err:.1e}")
    assert err < 1e-11
