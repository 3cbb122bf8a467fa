"""The workload configurations beyond the single 24^3 x 48 solve, against the oracle:

  * the mixed batch of 32 right-hand sides over 8^4, 12^4 and 16^4 lattices (one gauge field
    per size, mu_j uniform in [0, 0.3]) solved in one multishift_solve call: every shifted
    system of every problem is checked with the oracle's operator, and one 12^4 and one 16^4
    problem of the stored-basis batch equal the oracle's multishift BiCG;
  * restarted FOM-LR on 16^4 (mu = 0.2, 16 poles, k_max = 40), FP64 and mixed precision,
    equal to the oracle's restarted FOM-LR (the algorithm "Restarted FOM-LR")."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, krylov, rational

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

ALPHA, BETA = 0.1, 2.6
MIXED = dict(prec=sgn.F32_H16, theta32=1e-2, theta16=1e-5, delta=0.05)


def _rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c4():
    fields, plist = synth.mixed_batch_recipe(32)
    lats = [lattice(U, dims) for dims, U in fields]
    rf = sgn.sgn_rational_neuberger(16, ALPHA, BETA)
    om, sg, c = rational.coefficients(16, ALPHA, BETA)
    return fields, plist, lats, rf, (om, sg, c)


@pytest.mark.timeout(600)
def test_c4_every_shifted_system_of_every_problem(c4):
    """One call, 32 problems, per-shift solutions returned (mixed precision, tolerance 1e-10,
    verify: only the seed is reliable-updated, so every shifted system is checked in FP64 and
    refined where it is above the tolerance): ||y - (c^2 H^2 - sigma_i) x_i|| / ||y|| with the
    oracle's operator for all 16 x 32 systems."""
    fields, plist, lats, rf, (om, sg, c) = c4
    probs, xs_all, xs_dev = [], [], []
    for fi, mu, b in plist:
        bd = dev(b.ravel())
        xst = [torch.empty_like(bd) for _ in range(rf.s)]
        probs.append(sgn.Problem(lats[fi], mu, bd, torch.empty_like(bd), None, xst))
        xs_dev.append(xst)
    st = sgn.multishift_solve(probs, rf, tol=1e-10, verify=True, **MIXED)
    worst = 0.0
    for j, (fi, mu, b) in enumerate(plist):
        dims, U = fields[fi]
        W = WilsonRef(U, dims, 0.2)
        y = c * W.apply(b.ravel(), mu).ravel()
        ny = np.linalg.norm(y)
        xs = [host(t).ravel() for t in xs_dev[j]]
        res = [np.linalg.norm(y - (c * c * W.apply(W.apply(xi, mu), mu).ravel() - q * xi)) / ny
               for xi, q in zip(xs, sg)]
        worst = max(worst, max(res))
        assert _rel(host(probs[j].x), om @ np.stack(xs)) < 1e-12, j
        assert max(res) < 2e-10, (j, dims, mu, res)
    its = [s["iterations"] for s in st]
    ref_its = sum(s["refine_iterations"] for s in st)
    print(f"C4 per-shift batch: iterations {min(its)}..{max(its)}, refinement iterations {ref_its}, worst "
          f"oracle residual over 512 systems {worst:.2e}", flush=True)


@pytest.mark.timeout(600)  # the oracle's multishift BiCG on 16^4 takes about a minute
@pytest.mark.parametrize("j", [1, 2])
def test_c4_stored_basis_batch_against_oracle(c4, j):
    """The stored-basis batch (the timed form): problem 1 lives on 12^4, problem 2 on 16^4; each
    equals the oracle's multishift BiCG on the same 16-pole function."""
    fields, plist, lats, rf, (om, sg, c) = c4
    probs = []
    for fi, mu, b in plist:
        bd = dev(b.ravel())
        probs.append(sgn.Problem(lats[fi], mu, bd, torch.empty_like(bd)))
    sgn.multishift_solve(probs, rf, tol=1e-10, **MIXED)
    fi, mu, b = plist[j]
    dims, U = fields[fi]
    assert dims == ((12,) * 4 if j == 1 else (16,) * 4)
    W = WilsonRef(U, dims, 0.2)
    ref = krylov.multishift_bicg(lambda v: W.apply(v, mu), lambda v: W.apply_adj(v, mu), b.ravel(), om, sg, c,
                                 tol=1e-11)
    e = _rel(host(probs[j].x), ref)
    print(f"C4 problem {j} ({dims}, mu={mu:.3f}): stored-basis batch vs oracle {e:.2e}", flush=True)
    assert e < 1e-8


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32_H16])
def test_c3_fom_16x4_against_oracle(prec):
    dims = (16, 16, 16, 16)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    alpha, beta = 0.12, 2.6
    rf = sgn.sgn_rational_neuberger(16, alpha, beta)
    om, sg, c = rational.coefficients(16, alpha, beta)
    W = WilsonRef(U, dims, 0.2)
    bd = dev(b)
    x = torch.empty_like(bd)
    kw = dict(theta32=1e-2, theta16=1e-5) if prec != sgn.F64 else {}
    st = sgn.sign_arnoldi_rational(lattice(U, dims), 0.2, bd, x, rf, kmax=40, tol=1e-10, prec=prec, **kw)
    xo, info = krylov.fom_rational(lambda v: W.apply(v, 0.2), b, om, sg, c, 40, tol=1e-11, return_info=True)
    e = _rel(host(x), xo)
    print(f"C3 16^4 FOM k_max=40 prec={prec}: {st['restarts']} cycles (oracle {info['cycles']}), vs oracle "
          f"{e:.2e}", flush=True)
    assert e < 1e-8
