"""Parity of the HIP restarted GMRES-LR (sign_gmres_rational) with the oracle."""
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


def _gmres(lat, mu, b, rf, **kw):
    bd = dev(b)
    x = torch.empty_like(bd)
    st = sgn.sign_gmres_rational(lat, mu, bd, x, rf, **kw)
    return host(x).ravel(), st


def _deflated_case(s):
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
    om, sg, c = rational.coefficients(s, alpha, beta)
    target = krylov.deflation_xP(Lr.T, Rr.T, lm, b) + dense.rational_dense(H, krylov.project_out(Lr.T, Rr.T, b),
                                                                             om, sg, c)
    return dims, U, b, (Lr, Rr, lm), sgn.sgn_rational_neuberger(s, alpha, beta), target


@pytest.mark.parametrize("kmax", [10, 30])
def test_c1_gmres_matches_dense_rational(kmax):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    x, st = _gmres(lattice(U, dims), 0.3, b, rf, kmax=kmax, tol=1e-11)
    e = _rel(x, g["g16_b"])
    print(f"C1 GMRES kmax={kmax}: vs dense g16 {e:.2e}, cycles {st['restarts']}, matvecs {st['matvecs']}, "
          f"max res {st['residual']:.1e}", flush=True)
    assert e < 1e-8


def test_8x4_gmres_against_oracle():
    """Whole solve and cycle count against the oracle's GMRES-LR on an 8^4 lattice."""
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    W = WilsonRef(U, dims, 0.2)
    om, sg, c = rational.coefficients(16, 0.15, 2.6)
    rf = sgn.sgn_rational_neuberger(16, 0.15, 2.6)
    x, st = _gmres(lattice(U, dims), 0.2, b, rf, kmax=40, tol=1e-11)
    xo, info = krylov.gmres_rational(lambda v: W.apply(v, 0.2), b, om, sg, c, 40, tol=1e-11, return_info=True)
    e = _rel(x, xo)
    print(f"8^4 GMRES kmax=40: vs oracle {e:.2e}, cycles {st['restarts']} (oracle {info['cycles']}), "
          f"{st['krylov_ms']:.1f} ms", flush=True)
    assert e < 1e-8
    assert abs(st["restarts"] - info["cycles"]) <= 1


def test_gmres_shift_residuals_match_oracle_cycle_by_cycle():
    """After the same number of cycles, the collinearity factors rho_i times the
    seed residual norm agree with the oracle's for every shift (the small least
    squares and bordered solves of each cycle)."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    W = WilsonRef(U, dims, 0.2)
    om, sg, c = rational.coefficients(12, 0.2, 2.4)
    rf = sgn.sgn_rational_neuberger(12, 0.2, 2.4)
    _, st = _gmres(lattice(U, dims), 0.3, b, rf, kmax=8, tol=1e-4)
    _, info = krylov.gmres_rational(lambda v: W.apply(v, 0.3), b, om, sg, c, 8, max_cycles=st["restarts"],
                                    return_info=True)
    want = np.abs(info["rho"]) * info["seed_res"][-1] / info["ynorm"]
    got = np.asarray(st["shift_residual"][:12])
    print(f"GMRES {st['restarts']} cycles: shifted residuals {got.min():.2e}..{got.max():.2e}, "
          f"max rel diff {np.max(np.abs(got - want) / want):.1e}", flush=True)
    assert info["cycles"] == st["restarts"]
    assert np.max(np.abs(got - want) / want) < 1e-6
    assert got[info["seed"]] == pytest.approx(want[info["seed"]], rel=1e-6)


def test_gmres_and_fom_agree():
    dims = (4, 4, 4, 8)
    U = synth.gauge_field(dims, 0.45, 3)
    b = synth.gaussian_source(dims, 3).ravel()
    lat = lattice(U, dims)
    rf = sgn.sgn_rational_neuberger(14, 0.18, 2.5)
    xg, sg_ = _gmres(lat, 0.25, b, rf, kmax=24, tol=1e-11)
    bd = dev(b)
    xf = torch.empty_like(bd)
    sf = sgn.sign_arnoldi_rational(lat, 0.25, bd, xf, rf, kmax=24, tol=1e-11)
    e = _rel(xg, host(xf).ravel())
    print(f"GMRES vs FOM: {e:.2e}, cycles {sg_['restarts']} vs {sf['restarts']}", flush=True)
    assert e < 1e-9


def test_deflated_gmres_against_dense():
    dims, U, b, (Lr, Rr, lm), rf, target = _deflated_case(12)
    defl = sgn.Deflation(dev(Lr), dev(Rr), lm)
    x, st = _gmres(lattice(U, dims), 0.3, b, rf, defl=defl, kmax=12, tol=1e-12)
    e = _rel(x, target)
    print(f"deflated GMRES: vs dense {e:.2e}, cycles {st['restarts']}", flush=True)
    assert e < 1e-9


@pytest.mark.parametrize("prec", [sgn.F32, sgn.F32_H16])
def test_c1_mixed_gmres_matches_dense_rational(prec):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    g = np.load(GOLD)
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    x, st = _gmres(lattice(U, dims), 0.3, b, rf, kmax=20, tol=1e-10, prec=prec)
    e = _rel(x, g["g16_b"])
    print(f"C1 mixed GMRES prec={prec}: vs dense g16 {e:.2e}, cycles {st['restarts']} "
          f"({st['reliable_updates']} with the FP32 basis)", flush=True)
    assert st["reliable_updates"] >= 1
    assert e < 1e-8


def test_deflated_mixed_gmres():
    dims, U, b, (Lr, Rr, lm), rf, target = _deflated_case(16)
    defl = sgn.Deflation(dev(Lr), dev(Rr), lm)
    x, st = _gmres(lattice(U, dims), 0.3, b, rf, defl=defl, kmax=5, tol=1e-10, prec=sgn.F32)
    e = _rel(x, target)
    print(f"deflated mixed GMRES: vs dense {e:.2e}, cycles {st['restarts']} ({st['reliable_updates']} FP32)",
          flush=True)
    assert st["reliable_updates"] >= 1
    assert e < 1e-8


def test_gmres_zero_source_and_error_paths():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    lat = lattice(U, dims)
    rf = sgn.sgn_rational_neuberger(8, 0.2, 2.4)
    x, st = _gmres(lat, 0.3, np.zeros_like(b), rf, kmax=10)
    assert np.all(x == 0)
    with pytest.raises(sgn.SgnError) as e:
        _gmres(lat, 0.3, b, rf, kmax=10, prec=7)
    assert e.value.status == 1
    with pytest.raises(sgn.SgnError) as e:
        _gmres(lat, 0.3, b, rf, kmax=0)
    assert e.value.status == 1
    with pytest.raises(sgn.SgnError) as e:
        _gmres(lat, 0.3, b, rf, kmax=5, tol=1e-13, max_restarts=1)
    assert e.value.status == 5
