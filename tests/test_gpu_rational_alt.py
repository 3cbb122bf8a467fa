"""The rescaled Neuberger and Zolotarev approximations through the HIP solvers,
against the oracle's own coefficients and dense or Krylov evaluations."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, dense, krylov, rational

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402


def _rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _multishift(lat, mu, b, rf, **kw):
    bd = dev(b)
    x = torch.empty_like(bd)
    st = sgn.multishift_solve(sgn.Problem(lat, mu, bd, x), rf, **kw)[0]
    return host(x).ravel(), st


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32_H16])
def test_zolotarev_multishift_matches_oracle(prec):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 1)
    b = synth.gaussian_source(dims, 1).ravel()
    mu, n, alpha, beta = 0.1, 10, 0.2, 2.5
    rf, delta = sgn.sgn_rational_zolotarev(n, alpha, beta)
    om, sg, c, _ = rational.zolotarev(n, alpha, beta)
    W = WilsonRef(U, dims, 0.2)
    want = krylov.fom_rational(lambda v: W.apply(v, mu), b, om, sg, c, 40, tol=1e-12)
    x, st = _multishift(lattice(U, dims), mu, b, rf, tol=1e-11, prec=prec)
    e = _rel(x, want)
    print(f"Zolotarev n={n} (delta {delta:.1e}) multishift prec={prec}: vs oracle FOM {e:.2e}, "
          f"{st['iterations']} iterations", flush=True)
    assert e < 1e-8


def test_zolotarev_sign_within_uniform_bound_hermitian():
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 2)
    b = synth.gaussian_source(dims, 2).ravel()
    H = WilsonRef(U, dims, 0.2).dense(0.0)
    ev = np.abs(np.linalg.eigvalsh(H))
    alpha, beta = ev.min() * 0.999, ev.max() * 1.001
    want = dense.sign_herm(H, b)
    lat = lattice(U, dims)
    for n in (6, 12):
        rf, delta = sgn.sgn_rational_zolotarev(n, alpha, beta)
        x, st = _multishift(lat, 0.0, b, rf, tol=1e-12)
        e = _rel(x, want)
        print(f"Zolotarev n={n}: |g(H)b - sign(H)b|/|b| {e:.2e} <= delta {delta:.2e}", flush=True)
        assert e <= delta * (1 + 1e-6) + 1e-10


def test_rescaled_neuberger_through_fom_and_multishift():
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    mu, s, alpha, beta = 0.3, 12, 0.2, 2.6
    H = WilsonRef(U, dims, 0.2).dense(mu)
    rf, err = sgn.sgn_rational_neuberger_rescaled(s, alpha, beta)
    om, sg, c, e_max = rational.neuberger_rescaled(s, alpha, beta)
    want = dense.rational_dense(H, b, om, sg, c)
    lat = lattice(U, dims)
    x, _ = _multishift(lat, mu, b, rf, tol=1e-12)
    assert _rel(x, want) < 1e-9
    bd = dev(b)
    xf = torch.empty_like(bd)
    sgn.sign_arnoldi_rational(lat, mu, bd, xf, rf, kmax=20, tol=1e-12)
    assert _rel(host(xf), want) < 1e-9
    # the plain function differs from the rescaled one by the factor 1 + err
    rf0 = sgn.sgn_rational_neuberger(s, alpha, beta)
    x0, _ = _multishift(lat, mu, b, rf0, tol=1e-12)
    assert _rel(x, (1 + err) * x0) < 1e-9
