"""Batched multishift_solve: many problems (own lattice, mu, source) in one call.

All problems iterate in lockstep with one launch per step; the results must be
those of the one-problem solves, and on 8^4 lattices those of the oracle's
multishift BiCG on the same 16-pole function.
"""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, krylov, rational

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

ALPHA, BETA = 0.1, 2.6


def _rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solve(problems, rf, **kw):
    probs, outs = [], []
    for lat, mu, b in problems:
        bd = dev(np.ascontiguousarray(b).ravel())
        x = torch.empty_like(bd)
        probs.append(sgn.Problem(lat, mu, bd, x))
        outs.append(x)
    st = sgn.multishift_solve(probs, rf, **kw)
    return [host(x).ravel() for x in outs], st


def _small_set():
    out = []
    for dims, seed, mu in (((4, 4, 4, 4), 0, 0.3), ((4, 6, 4, 8), 1, 0.1), ((8, 8, 8, 8), 2, 0.25)):
        U = synth.gauge_field(dims, 0.4, seed)
        out.append((lattice(U, dims), mu, synth.gaussian_source(dims, seed)))
    return out


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32_H16])
def test_batch_equals_single_solves(prec):
    rf = sgn.sgn_rational_neuberger(16, ALPHA, BETA)
    probs = _small_set()
    xb, sb = _solve(probs, rf, tol=1e-10, prec=prec, poll=4)
    for k, p in enumerate(probs):
        xs, ss = _solve([p], rf, tol=1e-10, prec=prec, poll=4)
        e = _rel(xb[k], xs[0])
        print(f"prec={prec} problem {k}: batch vs single {e:.2e}, iterations {sb[k]['iterations']} / "
              f"{ss[0]['iterations']}", flush=True)
        assert sb[k]["iterations"] == ss[0]["iterations"]
        assert e < 1e-13


def test_batch_mixes_forms_and_zero_source():
    """A batch holding a stored-basis problem, a per-shift problem (x_shift) and a
    zero right-hand side."""
    rf = sgn.sgn_rational_neuberger(16, ALPHA, BETA)
    (la, mua, ba), (lb, mub, bb), (lc, muc, bc) = _small_set()
    xa = torch.empty(ba.size, dtype=torch.complex128, device="cuda")
    xb = torch.empty_like(xa)
    xsb = [torch.empty(bb.size, dtype=torch.complex128, device="cuda") for _ in range(rf.s)]
    xbb = torch.empty_like(xsb[0])
    zc = torch.zeros(bc.size, dtype=torch.complex128, device="cuda")
    xc = torch.full_like(zc, 7.0)
    st = sgn.multishift_solve([sgn.Problem(la, mua, dev(ba.ravel()), xa),
                               sgn.Problem(lb, mub, dev(bb.ravel()), xbb, None, xsb),
                               sgn.Problem(lc, muc, zc, xc)], rf, tol=1e-10, prec=sgn.F32_H16)
    assert np.all(host(xc) == 0)
    ya, _ = _solve([(la, mua, ba)], rf, tol=1e-10, prec=sgn.F64)
    yb, _ = _solve([(lb, mub, bb)], rf, tol=1e-10, prec=sgn.F64)
    ea, eb = _rel(host(xa), ya[0]), _rel(host(xbb), yb[0])
    comb = sum(w * host(t).ravel() for w, t in zip(list(rf.omega)[:rf.s], xsb))
    print(f"mixed batch vs FP64 singles: {ea:.2e} {eb:.2e}; per-shift sum {_rel(comb, yb[0]):.2e}", flush=True)
    assert ea < 1e-8 and eb < 1e-8
    assert _rel(comb, yb[0]) < 1e-8
    assert st[0]["iterations"] > 0 and st[1]["iterations"] > 0


def test_c4_mixed_batch_of_32():
    """32 right-hand sides over 8^4, 12^4 and 16^4 (one gauge field per size, mu_j in
    [0, 0.3]) in one call, mixed precision; the 8^4 ones against the oracle."""
    fields, plist = synth.mixed_batch_recipe(32)
    lats = [lattice(U, dims) for dims, U in fields]
    rf = sgn.sgn_rational_neuberger(16, ALPHA, BETA)
    probs = [(lats[fi], mu, b) for fi, mu, b in plist]
    x, st = _solve(probs, rf, tol=1e-10, prec=sgn.F32_H16)
    its = [s["iterations"] for s in st]
    print(f"C4 batch: iterations min {min(its)} max {max(its)}, max recurrence residual "
          f"{max(s['residual'] for s in st):.1e}", flush=True)
    assert max(s["residual"] for s in st) < 1e-10
    om, sg, c = rational.coefficients(16, ALPHA, BETA)
    for j in (0, 3):
        fi, mu, b = plist[j]
        dims, U = fields[fi]
        assert dims == (8, 8, 8, 8)
        W = WilsonRef(U, dims, 0.2)
        ref = krylov.multishift_bicg(lambda v: W.apply(v, mu), lambda v: W.apply_adj(v, mu), b.ravel(), om, sg, c,
                                     tol=1e-11)
        e = _rel(x[j], ref)
        print(f"C4 problem {j} (8^4, mu={mu:.3f}): vs oracle {e:.2e}", flush=True)
        assert e < 1e-8
    # every other problem: as its own FP64 solve
    for j in (1, 2, 4, 5):
        xs, _ = _solve([probs[j]], rf, tol=1e-11, prec=sgn.F64)
        e = _rel(x[j], xs[0])
        print(f"C4 problem {j} ({fields[plist[j][0]][0]}): batch mixed vs single FP64 {e:.2e}", flush=True)
        assert e < 1e-8


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32_H16])
def test_graph_replay_equals_plain_launches(prec):
    """Iterations replayed from a captured HIP graph (many replays, host work and
    reliable updates between them) give bit-identical results to plain launches."""
    rf = sgn.sgn_rational_neuberger(16, ALPHA, BETA)
    probs = _small_set()
    xg, sg = _solve(probs, rf, tol=1e-10, prec=prec, poll=3)
    xp, sp = _solve(probs, rf, tol=1e-10, prec=prec, poll=3, graph=False)
    for k in range(len(probs)):
        print(f"prec={prec} problem {k}: iterations {sg[k]['iterations']} / {sp[k]['iterations']}, "
              f"reliable updates {sg[k]['reliable_updates']}", flush=True)
        assert sg[k]["iterations"] == sp[k]["iterations"]
        assert np.array_equal(xg[k], xp[k])


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32_H16])
def test_bicgstab_lockstep_batch_equals_single_solves(prec):
    """multishift_bicgstab with several problems runs them in lockstep (one launch per step for all
    of them); each result equals its own single-problem solve to the tolerance's order, and the
    batch of problems on one lattice (multi-RHS stencil groups) gives the same as on separate ones."""
    rf = sgn.sgn_rational_neuberger(16, ALPHA, BETA)
    probs = _small_set()
    U = synth.gauge_field((8, 8, 8, 8), 0.4, 2)
    lat8 = lattice(U, (8, 8, 8, 8))
    probs += [(lat8, 0.1, synth.gaussian_source((8, 8, 8, 8), 7)), (lat8, 0.3, synth.gaussian_source((8, 8, 8, 8), 8))]
    kw = dict(tol=1e-10, prec=prec, poll=4)
    if prec != sgn.F64:
        kw.update(theta32=1e-2, theta16=1e-5, delta=0.05)
    outs, bprobs = [], []
    for lat, mu, b in probs:
        bd = dev(np.ascontiguousarray(b).ravel())
        x = torch.empty_like(bd)
        bprobs.append(sgn.Problem(lat, mu, bd, x))
        outs.append(x)
    sb = sgn.multishift_bicgstab(bprobs, rf, **kw)
    for k, (lat, mu, b) in enumerate(probs):
        bd = dev(np.ascontiguousarray(b).ravel())
        xs = torch.empty_like(bd)
        ss = sgn.multishift_bicgstab(sgn.Problem(lat, mu, bd, xs), rf, **kw)[0]
        e = _rel(host(outs[k]), host(xs))
        print(f"prec={prec} problem {k}: batch vs single {e:.2e}, iterations {sb[k]['iterations']} / "
              f"{ss['iterations']}, reliable updates {sb[k]['reliable_updates']} / {ss['reliable_updates']}",
              flush=True)
        assert e < (1e-9 if prec == sgn.F64 else 1e-8)
        assert abs(sb[k]["iterations"] - ss["iterations"]) <= max(2, ss["iterations"] // 10)


def test_bicgstab_lockstep_c4_against_oracle():
    """The 32 right-hand sides over 8^4 / 12^4 / 16^4 through the lockstep BiCGStab batch (mixed
    precision, every shifted system verified in FP64): the 8^4 problems against the oracle's
    multishift BiCGStab."""
    fields, plist = synth.mixed_batch_recipe(32)
    lats = [lattice(U, dims) for dims, U in fields]
    rf = sgn.sgn_rational_neuberger(16, ALPHA, BETA)
    om, sg, c = rational.coefficients(16, ALPHA, BETA)
    probs, outs = [], []
    for fi, mu, b in plist:
        bd = dev(b.ravel())
        x = torch.empty_like(bd)
        probs.append(sgn.Problem(lats[fi], mu, bd, x))
        outs.append(x)
    st = sgn.multishift_bicgstab(probs, rf, tol=1e-10, prec=sgn.F32_H16, theta32=1e-2, theta16=1e-5, delta=0.05,
                                 verify=True)
    its = [s["iterations"] for s in st]
    print(f"C4 BiCGStab lockstep: iterations {min(its)}..{max(its)}, verified shifted residuals <= "
          f"{max(s['residual'] for s in st):.1e}", flush=True)
    assert max(s["residual"] for s in st) <= 1e-10
    for j in (0, 3, 6):
        fi, mu, b = plist[j]
        dims, U = fields[fi]
        assert dims == (8, 8, 8, 8)
        W = WilsonRef(U, dims, 0.2)
        ref = krylov.multishift_bicgstab(lambda v: W.apply(v, mu), b.ravel(), om, sg, c, tol=1e-11)
        e = _rel(host(outs[j]), ref)
        print(f"C4 problem {j}: lockstep BiCGStab vs oracle {e:.2e}", flush=True)
        assert e < 1e-9


@pytest.mark.parametrize("solver", ["bicg", "bicgstab", "qmr"])
def test_lockstep_batches_with_deflated_problems(solver):
    """A batch mixing deflated problems (each its own deflation set, on two lattices) with an
    undeflated one: every result equals the dense target x_P + g(cH)(I - P) b (Eq. exact_proj)."""
    from oracle import dense
    cases = []
    for dims, seed, mu in (((2, 2, 2, 4), 0, 0.3), ((2, 2, 4, 4), 1, 0.2)):
        U = synth.gauge_field(dims, 0.5, seed)
        H = WilsonRef(U, dims, 0.2).dense(mu)
        lam, R = np.linalg.eig(H)
        Linv = np.linalg.inv(R)
        idx = np.argsort(np.abs(lam.real))[:8]
        cases.append((U, dims, mu, H, Linv[idx].conj(), R[:, idx].T.copy(), lam[idx]))
    alpha = 0.15
    beta = max(float(np.abs(np.linalg.eigvals(c[3])).max()) for c in cases)
    rf = sgn.sgn_rational_neuberger(14, alpha, beta)
    om, sg, c = rational.coefficients(14, alpha, beta)
    probs, outs, targets, keep = [], [], [], []
    for k, (U, dims, mu, H, Lr, Rr, lm) in enumerate(cases):
        lat = lattice(U, dims)
        for j, deflate in enumerate((True, False) if k == 0 else (True,)):
            b = synth.gaussian_source(dims, 10 + 3 * k + j).ravel()
            bd = dev(b)
            x = torch.empty_like(bd)
            defl = sgn.Deflation(dev(Lr), dev(Rr), lm) if deflate else None
            keep.append(defl)
            probs.append(sgn.Problem(lat, mu, bd, x, defl))
            outs.append(x)
            if deflate:
                t = krylov.deflation_xP(Lr.T, Rr.T, lm, b) + dense.rational_dense(
                    H, krylov.project_out(Lr.T, Rr.T, b), om, sg, c)
            else:
                t = dense.rational_dense(H, b, om, sg, c)
            targets.append(t)
    kw = dict(tol=1e-12)
    f = {"bicg": sgn.multishift_solve, "bicgstab": sgn.multishift_bicgstab, "qmr": sgn.multishift_qmr}[solver]
    st = f(probs, rf, **kw)
    for k, (x, t) in enumerate(zip(outs, targets)):
        e = _rel(host(x), t)
        print(f"{solver} problem {k}: vs dense target {e:.2e}, {st[k]['iterations']} iterations", flush=True)
        assert e < 1e-9
