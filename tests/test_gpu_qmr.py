"""Parity of the HIP multishift QMR (multishift_qmr) with the oracle."""
import os

import numpy as np
import pytest

import synth
from oracle import WilsonRef, dense, krylov, rational

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_dense.npz")


def _rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solve(lat, mu, b, rf, defl=None, want_shifts=False, **kw):
    bd = dev(b)
    x = torch.empty_like(bd)
    xs = [torch.empty_like(bd) for _ in range(rf.s)] if want_shifts else None
    st = sgn.multishift_qmr(sgn.Problem(lat, mu, bd, x, defl, xs), rf, **kw)[0]
    if want_shifts:
        return host(x).ravel(), st, [host(t).ravel() for t in xs]
    return host(x).ravel(), st


def test_c1_qmr_matches_dense_rational():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    lat = lattice(U, dims)
    x, st = _solve(lat, 0.3, b, rf, tol=1e-11)
    e = _rel(x, g["g16_b"])
    bd = dev(b)
    xb = torch.empty_like(bd)
    sb = sgn.multishift_solve(sgn.Problem(lat, 0.3, bd, xb), rf, tol=1e-11)[0]
    print(f"C1 QMR: vs dense g16 {e:.2e}, {st['iterations']} iterations ({st['matvecs']} matvecs); "
          f"BiCG {sb['iterations']} iterations, QMR vs BiCG {_rel(x, host(xb)):.1e}", flush=True)
    assert e < 1e-8
    assert _rel(x, host(xb)) < 1e-8


def test_8x4_qmr_against_oracle_same_steps():
    """The oracle runs exactly the GPU's number of Lanczos steps; x and every x_i agree."""
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    W = WilsonRef(U, dims, 0.2)
    om, sg, c = rational.coefficients(16, 0.15, 2.6)
    rf = sgn.sgn_rational_neuberger(16, 0.15, 2.6)
    x, st, xs = _solve(lattice(U, dims), 0.2, b, rf, want_shifts=True, tol=1e-11)
    k = st["iterations"]
    xo, info = krylov.multishift_qmr(lambda v: W.apply(v, 0.2), lambda v: W.apply_adj(v, 0.2), b, om, sg, c,
                                     k=k, return_info=True)
    e = _rel(x, xo)
    worst = max(_rel(xs[i], info["X"][i]) for i in range(16))
    tau_gpu = np.array(st["shift_residual"][:16])
    tau_or = info["tau"] / info["ynorm"]
    print(f"8^4 QMR: {k} steps, {st['krylov_ms']:.1f} ms; vs oracle x {e:.2e}, worst x_i {worst:.2e}; "
          f"max tau {tau_gpu.max():.2e} (oracle {tau_or.max():.2e})", flush=True)
    assert e < 1e-8
    assert worst < 1e-8
    assert np.all(tau_gpu <= 1e-11)
    assert tau_or.max() <= 1e-10


def test_qmr_verified_residuals_and_bound():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 2)
    b = synth.gaussian_source(dims, 2).ravel()
    W = WilsonRef(U, dims, 0.2)
    rf = sgn.sgn_rational_neuberger(10, 0.2, 2.4)
    om, sg, c = rational.coefficients(10, 0.2, 2.4)
    x, st, xs = _solve(lattice(U, dims), 0.25, b, rf, want_shifts=True, tol=1e-10, verify=True)
    k = st["iterations"]
    y = c * W.apply(b, 0.25).ravel()
    for i in range(10):
        Ax = W.apply(W.apply(xs[i], 0.25), 0.25).ravel()
        res = np.linalg.norm(y - (c * c * Ax - sg[i] * xs[i])) / np.linalg.norm(y)
        assert res == pytest.approx(st["shift_residual"][i], rel=1e-3, abs=1e-14)
        assert res <= np.sqrt(k + 1) * 1e-10
    assert _rel(x, om @ np.stack(xs)) < 1e-12
    print(f"QMR verified residuals: {k} steps, max {st['residual']:.2e}", flush=True)


def test_deflated_qmr_against_dense():
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    H = WilsonRef(U, dims, 0.2).dense(0.3)
    lam, R = np.linalg.eig(H)
    Linv = np.linalg.inv(R)
    idx = np.argsort(np.abs(lam.real))[:8]
    Lr, Rr, lm = Linv[idx].conj(), R[:, idx].T.copy(), lam[idx]
    rest = np.delete(lam, idx)
    alpha, beta = float(np.abs(rest).min()), float(np.abs(lam).max())
    om, sg, c = rational.coefficients(12, alpha, beta)
    rf = sgn.sgn_rational_neuberger(12, alpha, beta)
    defl = sgn.Deflation(dev(Lr), dev(Rr), lm)
    x, st = _solve(lattice(U, dims), 0.3, b, rf, defl=defl, tol=1e-12)
    target = krylov.deflation_xP(Lr.T, Rr.T, lm, b) + dense.rational_dense(H, krylov.project_out(Lr.T, Rr.T, b),
                                                                             om, sg, c)
    print(f"deflated QMR: {st['iterations']} steps, vs dense {_rel(x, target):.1e}", flush=True)
    assert _rel(x, target) < 1e-9


@pytest.mark.parametrize("prec", [sgn.F32, sgn.F32_H16])
def test_c1_mixed_qmr_matches_dense_rational(prec):
    """Mixed schedule: FP64 steps until tau < 1e-3 ||y||, then the FP32 stencil (FP16 links below
    1e-6 ||y||) with FP64 recurrences."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    x, st = _solve(lattice(U, dims), 0.3, b, rf, tol=1e-11, prec=prec, verify=True)
    e = _rel(x, g["g16_b"])
    print(f"C1 mixed QMR prec={prec}: vs dense g16 {e:.2e}, {st['iterations']} steps, "
          f"max true residual {st['residual']:.1e}", flush=True)
    assert e < 1e-8


def test_8x4_mixed_qmr_against_oracle():
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    W = WilsonRef(U, dims, 0.2)
    om, sg, c = rational.coefficients(16, 0.15, 2.6)
    rf = sgn.sgn_rational_neuberger(16, 0.15, 2.6)
    x, st = _solve(lattice(U, dims), 0.2, b, rf, tol=1e-11, prec=sgn.F32_H16, theta32=1e-2, theta16=1e-5)
    xo = krylov.multishift_qmr(lambda v: W.apply(v, 0.2), lambda v: W.apply_adj(v, 0.2), b, om, sg, c,
                               tol=1e-11, check_every=8)
    e = _rel(x, xo)
    print(f"8^4 mixed QMR (1e-2, 1e-5): vs oracle {e:.2e}, {st['iterations']} steps, {st['total_ms']:.1f} ms",
          flush=True)
    assert e < 1e-8


def test_qmr_zero_source_and_errors():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    lat = lattice(U, dims)
    rf = sgn.sgn_rational_neuberger(8, 0.2, 2.4)
    x, st = _solve(lat, 0.3, np.zeros_like(b), rf)
    assert np.all(x == 0) and st["iterations"] == 0
    with pytest.raises(sgn.SgnError) as e:
        _solve(lat, 0.3, b, rf, tol=1e-11, maxiter=3)
    assert e.value.status == 5
    with pytest.raises(sgn.SgnError) as e:
        _solve(lat, 0.3, b, rf, basis_slots=-1)
    assert e.value.status == 1
    with pytest.raises(sgn.SgnError) as e:
        _solve(lat, 0.3, b, rf, basis_slots=9)  # stored basis beyond its cap
    assert e.value.status == 3


def test_full_size_qmr_residuals_with_oracle_operator():
    """24^3 x 48, 16 poles, tolerance 1e-9 on the quasi-residual: all shifted solutions
    satisfy their systems (checked with the oracle's operator on the CPU)."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    alpha, beta = 0.12, 2.6
    rf = sgn.sgn_rational_neuberger(16, alpha, beta)
    om, sg, c = rational.coefficients(16, alpha, beta)
    x, st, xs = _solve(lattice(U, dims), 0.2, b, rf, want_shifts=True, tol=1e-9)
    k = st["iterations"]
    print(f"24^3x48 QMR: {k} steps, {st['krylov_ms']:.0f} ms", flush=True)
    W = WilsonRef(U, dims, 0.2)
    y = c * W.apply(b, 0.2).ravel()
    for i in range(rf.s):  # every shifted system
        Ax = W.apply(W.apply(xs[i], 0.2), 0.2).ravel()
        res = np.linalg.norm(y - (c * c * Ax - sg[i] * xs[i])) / np.linalg.norm(y)
        print(f"  shift {i}: oracle residual {res:.2e}, quasi-residual {st['shift_residual'][i]:.2e}", flush=True)
        assert res < np.sqrt(k + 1) * 1e-9
    assert _rel(x, om @ np.stack(xs)) < 1e-12


def test_qmr_on_a_side_stream_matches_default_stream():
    """The solve, its per-shift lifts and the verification on a non-default stream give the same
    bits as on the default stream."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 3)
    b = synth.gaussian_source(dims, 3).ravel()
    lat = lattice(U, dims)
    rf = sgn.sgn_rational_neuberger(10, 0.2, 2.4)
    x0, st0, xs0 = _solve(lat, 0.25, b, rf, want_shifts=True, tol=1e-10, verify=True)
    side = torch.cuda.Stream()
    bd = dev(b)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        x = torch.empty_like(bd)
        xs = [torch.empty_like(bd) for _ in range(rf.s)]
        st = sgn.multishift_qmr(sgn.Problem(lat, 0.25, bd, x, None, xs), rf, tol=1e-10, verify=True,
                                stream=side)[0]
    side.synchronize()
    assert np.array_equal(host(x).ravel(), x0)
    for i in range(rf.s):
        assert np.array_equal(host(xs[i]).ravel(), xs0[i])
    assert st["iterations"] == st0["iterations"] and st["shift_residual"] == st0["shift_residual"]


def test_qmr_two_problems_in_one_call():
    """Problems of one call (different mu and sources on one lattice) run in lockstep (their stencils
    as one multi-RHS launch) and give the same bits as separate calls; stats come back per problem."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    lat = lattice(U, dims)
    rf = sgn.sgn_rational_neuberger(12, 0.2, 2.4)
    cases = [(0.3, synth.gaussian_source(dims, 4).ravel()), (0.1, synth.gaussian_source(dims, 5).ravel())]
    single = [_solve(lat, mu, b, rf, tol=1e-10) for mu, b in cases]
    bds = [dev(b) for _, b in cases]
    xs = [torch.empty_like(t) for t in bds]
    sts = sgn.multishift_qmr([sgn.Problem(lat, mu, bd, x) for (mu, _), bd, x in zip(cases, bds, xs)], rf,
                             tol=1e-10)
    assert len(sts) == 2
    for k in range(2):
        assert np.array_equal(host(xs[k]).ravel(), single[k][0])
        assert sts[k]["iterations"] == single[k][1]["iterations"]


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32_H16])
def test_qmr_lockstep_batch_of_uneven_lattices(prec):
    """Problems on lattices of different sizes (and two on one lattice) in one call: each result
    equals its own single-problem solve to the tolerance's order with the same number of steps (to
    within two), and the 8^4 ones equal the oracle's multishift QMR."""
    rf = sgn.sgn_rational_neuberger(16, 0.1, 2.6)
    om, sg, c = rational.coefficients(16, 0.1, 2.6)
    cases = []
    for dims, seed, mu in (((4, 4, 4, 4), 0, 0.3), ((4, 6, 4, 8), 1, 0.1), ((8, 8, 8, 8), 2, 0.25)):
        U = synth.gauge_field(dims, 0.4, seed)
        cases.append((U, dims, lattice(U, dims), mu, synth.gaussian_source(dims, seed).ravel()))
    U8, d8, l8 = cases[2][:3]
    cases.append((U8, d8, l8, 0.05, synth.gaussian_source(d8, 9).ravel()))
    kw = dict(tol=1e-10, prec=prec, poll=4)
    if prec != sgn.F64:
        kw.update(theta32=1e-3, theta16=1e-6)
    bds = [dev(b) for *_, b in cases]
    xs = [torch.empty_like(t) for t in bds]
    sts = sgn.multishift_qmr([sgn.Problem(lat, mu, bd, x) for (_, _, lat, mu, _), bd, x in zip(cases, bds, xs)],
                             rf, **kw)
    for k, (U, dims, lat, mu, b) in enumerate(cases):
        xk, sk = _solve(lat, mu, b, rf, **kw)
        e = _rel(host(xs[k]), xk)
        print(f"prec={prec} problem {k} {dims}: batch vs single {e:.2e}, steps {sts[k]['iterations']} / "
              f"{sk['iterations']}", flush=True)
        assert e < (1e-11 if prec == sgn.F64 else 1e-8)
        assert abs(sts[k]["iterations"] - sk["iterations"]) <= 2
        if dims == (8, 8, 8, 8):
            W = WilsonRef(U, dims, 0.2)
            ref = krylov.multishift_qmr(lambda v: W.apply(v, mu), lambda v: W.apply_adj(v, mu), b, om, sg, c,
                                        tol=1e-11)
            eo = _rel(host(xs[k]), ref)
            print(f"   vs oracle {eo:.2e}", flush=True)
            assert eo < (1e-9 if prec == sgn.F64 else 1e-8)


def test_qmr_batch_with_a_zero_source():
    """A zero right-hand side inside a lockstep QMR batch gives x = 0 and leaves the other problem
    as its single solve."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    lat = lattice(U, dims)
    rf = sgn.sgn_rational_neuberger(12, 0.2, 2.4)
    b = synth.gaussian_source(dims, 4).ravel()
    xs, _ = _solve(lat, 0.3, b, rf, tol=1e-10)
    bd = dev(b)
    zd = torch.zeros_like(bd)
    x0, x1 = torch.full_like(bd, 3.0), torch.empty_like(bd)
    sgn.multishift_qmr([sgn.Problem(lat, 0.1, zd, x0), sgn.Problem(lat, 0.3, bd, x1)], rf, tol=1e-10)
    assert np.all(host(x0) == 0)
    assert _rel(host(x1), xs) < 1e-12
