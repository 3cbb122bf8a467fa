"""Parity of the HIP multishift BiCG-LR (multishift_solve) with the oracle.

The target of the rational path is g_s(cA)(I-P)b + x_P with the same 16-pole
Neuberger function the oracle evaluates; its distance to the true sign is a
property of the rational function (circle theorem), reported separately.
"""
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
    st = sgn.multishift_solve(sgn.Problem(lat, mu, bd, x, defl, xs), rf, **kw)[0]
    out = host(x).ravel()
    if want_shifts:
        return out, st, [host(t).ravel() for t in xs]
    return out, st


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_c1_multishift_matches_dense_rational(prec):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    lat = lattice(U, dims)
    x, st = _solve(lat, 0.3, b, rf, tol=1e-10, prec=prec, verify=True)
    e = _rel(x, g["g16_b"])
    print(f"C1 multishift prec={prec}: vs dense g16 {e:.2e}, vs sign {_rel(x, g['sign_b']):.2e}, "
          f"iters {st['iterations']}, reliable {st['reliable_updates']}, max shift res {st['residual']:.1e}",
          flush=True)
    assert e < 1e-8
    assert st["residual"] < 1e-9


def test_shift_solutions_match_oracle():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    alpha, beta = float(g["alpha"]), float(g["beta"])
    rf = sgn.sgn_rational_neuberger(16, alpha, beta)
    om, sg, c = rational.coefficients(16, alpha, beta)
    W = WilsonRef(U, dims, 0.2)
    lat = lattice(U, dims)
    x, st, xs = _solve(lat, 0.3, b, rf, want_shifts=True, tol=1e-11)
    _, info = krylov.multishift_bicg(lambda v: W.apply(v, 0.3), lambda v: W.apply_adj(v, 0.3), b, om, sg, c,
                                     tol=1e-11, return_info=True)
    for i in range(16):
        assert _rel(xs[i], info["X"][i]) < 1e-8, i


@pytest.mark.parametrize("mu", [0.0, 0.2])
def test_8x4_multishift_against_oracle(mu):
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    W = WilsonRef(U, dims, 0.2)
    alpha, beta = 0.15, 2.6          # a circle enclosing the spectrum for these fields
    om, sg, c = rational.coefficients(16, alpha, beta)
    rf = sgn.sgn_rational_neuberger(16, alpha, beta)
    lat = lattice(U, dims)
    xo = krylov.multishift_bicg(lambda v: W.apply(v, mu), lambda v: W.apply_adj(v, mu), b, om, sg, c, tol=1e-11)
    for prec in (sgn.F64, sgn.F32, sgn.F32_H16):
        x, st = _solve(lat, mu, b, rf, tol=1e-10, prec=prec)
        e = _rel(x, xo)
        print(f"8^4 mu={mu} prec={prec}: vs oracle {e:.2e} iters {st['iterations']} "
              f"reliable {st['reliable_updates']} {st['krylov_ms']:.1f} ms", flush=True)
        assert e < 1e-8


def test_deflated_multishift_against_oracle():
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    W = WilsonRef(U, dims, 0.2)
    H = W.dense(0.3)
    lam, R = np.linalg.eig(H)
    Linv = np.linalg.inv(R)
    idx = np.argsort(np.abs(lam.real))[:8]
    Lr, Rr, lm = Linv[idx].conj(), R[:, idx].T.copy(), lam[idx]
    rest = np.delete(lam, idx)
    alpha, beta = float(np.abs(rest).min()), float(np.abs(lam).max())
    om, sg, c = rational.coefficients(12, alpha, beta)
    rf = sgn.sgn_rational_neuberger(12, alpha, beta)
    lat = lattice(U, dims)
    defl = sgn.Deflation(dev(Lr), dev(Rr), lm)
    x, _ = _solve(lat, 0.3, b, rf, defl=defl, tol=1e-11)
    target = krylov.deflation_xP(Lr.T, Rr.T, lm, b) + dense.rational_dense(H, krylov.project_out(Lr.T, Rr.T, b),
                                                                             om, sg, c)
    assert _rel(x, target) < 1e-9


def test_two_problems_two_lattices_one_call():
    fields = [((4, 4, 4, 4), 0.5, 0, 0.3), ((4, 4, 6, 8), 0.4, 1, 0.1)]
    rf = sgn.sgn_rational_neuberger(12, 0.15, 2.6)
    om, sg, c = rational.coefficients(12, 0.15, 2.6)
    probs, refs, keep = [], [], []
    for dims, eps, seed, mu in fields:
        U = synth.gauge_field(dims, eps, seed)
        b = synth.gaussian_source(dims, seed).ravel()
        lat = lattice(U, dims)
        bd = dev(b)
        x = torch.empty_like(bd)
        keep += [lat, bd]
        probs.append(sgn.Problem(lat, mu, bd, x))
        W = WilsonRef(U, dims, 0.2)
        refs.append(krylov.multishift_bicg(lambda v, W=W, mu=mu: W.apply(v, mu),
                                           lambda v, W=W, mu=mu: W.apply_adj(v, mu), b, om, sg, c, tol=1e-11))
    sts = sgn.multishift_solve(probs, rf, tol=1e-10, prec=sgn.F32)
    for p, ref, st in zip(probs, refs, sts):
        assert _rel(host(p.x), ref) < 1e-8, st


def test_full_size_residuals_with_oracle_operator():
    """24^3 x 48, mixed precision with FP16 links: the returned shifted solutions
    satisfy their systems, checked with the oracle's own operator on the CPU."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    alpha, beta = 0.12, 2.6
    rf = sgn.sgn_rational_neuberger(16, alpha, beta)
    om, sg, c = rational.coefficients(16, alpha, beta)
    lat = lattice(U, dims)
    x, st, xs = _solve(lat, 0.2, b, rf, want_shifts=True, tol=1e-10, prec=sgn.F32_H16)
    print(f"24^3x48 mixed: iters {st['iterations']} reliable {st['reliable_updates']} "
          f"{st['krylov_ms']:.0f} ms", flush=True)
    W = WilsonRef(U, dims, 0.2)
    y = c * W.apply(b, 0.2).ravel()
    for i in range(rf.s):  # every shifted system
        Ax = W.apply(W.apply(xs[i], 0.2), 0.2).ravel()
        res = np.linalg.norm(y - (c * c * Ax - sg[i] * xs[i])) / np.linalg.norm(y)
        print(f"  shift {i}: oracle residual {res:.2e}", flush=True)
        assert res < 1e-9
    assert _rel(x, om @ np.stack(xs)) < 1e-12


def test_error_paths():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    lat = lattice(U, dims)
    b = synth.gaussian_source(dims, 0).ravel()
    rf = sgn.sgn_rational_neuberger(8, 0.2, 2.4)
    with pytest.raises(sgn.SgnError) as e:
        _solve(lat, 0.3, b, rf, tol=0.0)
    assert e.value.status == 1
    with pytest.raises(sgn.SgnError) as e:
        _solve(lat, 0.3, b, rf, tol=1e-12, maxiter=3)
    assert e.value.status == 5


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32_H16])
def test_stored_basis_equals_per_shift_vectors(prec):
    """The stored-basis form and the per-shift-vector form are the same iteration."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    lat = lattice(U, dims)
    xb, sb = _solve(lat, 0.3, b, rf, tol=1e-10, prec=prec)
    xe, se = _solve(lat, 0.3, b, rf, tol=1e-10, prec=prec, basis_slots=-1)
    print(f"prec={prec}: basis vs per-shift {_rel(xb, xe):.2e}; vs dense g16 {_rel(xb, g['g16_b']):.2e} / "
          f"{_rel(xe, g['g16_b']):.2e}; iterations {sb['iterations']} / {se['iterations']}", flush=True)
    # the update kernels round differently (FMA contraction), and BiCG turns ulp-level
    # differences into a few iterations more or less; the results agree to tolerance
    assert abs(sb["iterations"] - se["iterations"]) <= 0.1 * se["iterations"]
    assert _rel(xb, xe) < 1e-9
    assert _rel(xb, g["g16_b"]) < 1e-8 and _rel(xe, g["g16_b"]) < 1e-8


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_basis_budget_fallback(prec):
    """A basis budget smaller than the iteration count: the solver rebuilds p_i, x_i
    from the stored residuals mid-solve and finishes with per-shift vectors."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    lat = lattice(U, dims)
    for slots in (10, 37):
        x, st = _solve(lat, 0.3, b, rf, tol=1e-10, prec=prec, basis_slots=slots, poll=4)
        e = _rel(x, g["g16_b"])
        print(f"prec={prec} basis_slots={slots}: vs dense g16 {e:.2e}, iterations {st['iterations']}", flush=True)
        assert e < 1e-8


def test_verify_refines_shifted_systems_above_tolerance():
    """FP16 links from the first iteration leave the shifted systems far above the tolerance; with
    verify every one of them is refined in FP64 before the combination, and the result meets the
    FP64 target."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    lat = lattice(U, dims)
    coarse = dict(prec=sgn.F32_H16, theta32=1.0, theta16=1.0)
    x0, st0 = _solve(lat, 0.3, b, rf, tol=1e-10, **coarse)
    x, st = _solve(lat, 0.3, b, rf, tol=1e-10, verify=True, **coarse)
    e0, e = _rel(x0, g["g16_b"]), _rel(x, g["g16_b"])
    print(f"FP16 links throughout: error {e0:.1e} without refinement, {e:.1e} with "
          f"({st['refine_iterations']} refinement iterations, max shifted residual {st['residual']:.1e})",
          flush=True)
    assert st["refine_iterations"] > 0 and st0["refine_iterations"] == 0
    assert st["residual"] <= 1e-10
    assert e < 1e-8 < e0
