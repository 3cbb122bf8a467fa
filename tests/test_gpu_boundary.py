"""Error behaviour of the C ABI on the GPU: an inconsistent LR deflation set
(L^H R != I, section "Deflation") is refused by every solver, a shadow vector
orthogonal to the residual is reported as a two-sided Lanczos breakdown
(section on the two-sided Lanczos process), and the binding refuses tensors of
the wrong device, dtype, layout or size before anything is launched.  Every
error here is forced from the host; no kernel is made to fail."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, eigen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

DIMS = (2, 2, 2, 4)
MU = 0.3


def _setup(m=3):
    U = synth.gauge_field(DIMS, 0.5, 0)
    b = synth.gaussian_source(DIMS, 0).ravel()
    A = WilsonRef(U, DIMS, 0.2).dense(MU)
    L, R, lam = eigen.critical_eigenpairs(A, m)
    return U, b, L, R, lam


def _defl(L, R, lam):
    return sgn.Deflation(dev(np.ascontiguousarray(L.T)), dev(np.ascontiguousarray(R.T)), lam)


def _solvers(lat, b, defl, rf):
    bd = dev(b)
    x = torch.empty_like(bd)
    return {
        "sign_lanczos_2sided": lambda: sgn.sign_lanczos_2sided(lat, MU, bd, x, defl=defl, k=40),
        "sign_arnoldi_rational": lambda: sgn.sign_arnoldi_rational(lat, MU, bd, x, rf, defl=defl, kmax=20),
        "sign_gmres_rational": lambda: sgn.sign_gmres_rational(lat, MU, bd, x, rf, defl=defl, kmax=20),
        "multishift_solve": lambda: sgn.multishift_solve(sgn.Problem(lat, MU, bd, x, defl), rf),
        "multishift_bicgstab": lambda: sgn.multishift_bicgstab(sgn.Problem(lat, MU, bd, x, defl), rf),
        "multishift_qmr": lambda: sgn.multishift_qmr(sgn.Problem(lat, MU, bd, x, defl), rf),
    }


def test_consistent_deflation_set_is_accepted():
    U, b, L, R, lam = _setup()
    lat = lattice(U, DIMS)
    rf = sgn.sgn_rational_neuberger(16, 0.2, 2.6)
    for name, run in _solvers(lat, b, _defl(L, R, lam), rf).items():
        run()  # raises on any error


@pytest.mark.parametrize("kind", ["scaled", "permuted", "foreign"])
def test_inconsistent_deflation_set_is_refused(kind):
    """L^H R = I is what makes P = R L^H a projector; each solver must refuse a set
    that breaks it: one left vector scaled, left vectors in another order than the
    right ones, or left vectors of other eigenvalues."""
    U, b, L, R, lam = _setup()
    if kind == "scaled":
        L = L.copy()
        L[:, 1] *= 1.5
    elif kind == "permuted":
        L = L[:, [1, 0, 2]]
    else:
        A = WilsonRef(U, DIMS, 0.2).dense(MU)
        L2, _, _ = eigen.critical_eigenpairs(A, 6)
        L = L2[:, 3:6]
    print(f"{kind}: max |L^H R - I| = {np.abs(L.conj().T @ R - np.eye(3)).max():.2e}", flush=True)
    lat = lattice(U, DIMS)
    rf = sgn.sgn_rational_neuberger(16, 0.2, 2.6)
    for name, run in _solvers(lat, b, _defl(L, R, lam), rf).items():
        with pytest.raises(sgn.SgnError) as e:
            run()
        assert e.value.status == 1, (name, e.value)
        assert "L^H R" in str(e.value), (name, e.value)


def test_slightly_inexact_set_within_tolerance_is_accepted():
    """An eigensolver's set is biorthonormal only to its accuracy (1e-12 relative here)."""
    U, b, L, R, lam = _setup()
    rng = np.random.default_rng(3)
    L = L + 1e-12 * np.linalg.norm(L, axis=0) * (rng.standard_normal(L.shape) + 1j * rng.standard_normal(L.shape))
    lat = lattice(U, DIMS)
    bd = dev(b)
    x = torch.empty_like(bd)
    sgn.sign_lanczos_2sided(lat, MU, bd, x, defl=_defl(L, R, lam), k=40)


def test_shadow_orthogonal_to_residual_is_a_breakdown():
    """A one-vector set with L^H R = 1 built so that the shadow residual (I - L R^H) b is
    orthogonal to the residual (I - R L^H) b while neither is zero: r a unit vector,
    l = r + b_perp / (r^H b) + w with b_perp the part of b orthogonal to r and w a unit vector
    orthogonal to r and b.  Then (I - L R^H) b = -(r^H b) w and r^H-products cancel exactly."""
    U = synth.gauge_field(DIMS, 0.5, 0)
    b = synth.gaussian_source(DIMS, 0).ravel()
    rng = np.random.default_rng(11)
    z = rng.standard_normal(b.size) + 1j * rng.standard_normal(b.size)
    r = b + 0.7 * z / np.linalg.norm(z)
    r /= np.linalg.norm(r)
    a = np.vdot(r, b)
    bp = b - r * a
    w = rng.standard_normal(b.size) + 1j * rng.standard_normal(b.size)
    for v in (r, bp / np.linalg.norm(bp)):
        w -= v * np.vdot(v, w)
    w /= np.linalg.norm(w)
    ell = r + bp / a + w
    res = b - r * np.vdot(ell, b)
    shadow = b - ell * a
    assert abs(np.vdot(ell, r) - 1) < 1e-13
    assert np.linalg.norm(res) > 0.1 and np.linalg.norm(shadow) > 0.1
    assert abs(np.vdot(res, shadow)) < 1e-14 * np.linalg.norm(res) * np.linalg.norm(shadow)
    lat = lattice(U, DIMS)
    defl = _defl(ell[:, None], r[:, None], np.array([1.0 + 0.0j]))
    bd = dev(b)
    x = torch.empty_like(bd)
    with pytest.raises(sgn.SgnError) as e:
        sgn.sign_lanczos_2sided(lat, MU, bd, x, defl=defl, k=40)
    assert e.value.status == 4, e.value  # SGN_ERR_BREAKDOWN
    print(f"breakdown reported: {e.value}", flush=True)


def test_binding_refuses_bad_device_tensors():
    U = synth.gauge_field(DIMS, 0.5, 0)
    b = synth.gaussian_source(DIMS, 0).ravel()
    lat = lattice(U, DIMS)
    n = b.size
    good = dev(b)
    out = torch.empty_like(good)
    rf = sgn.sgn_rational_neuberger(16, 0.2, 2.6)
    bad = {
        "complex64": good.to(torch.complex64),
        "short": good[: n - 12].clone(),
        "strided": torch.empty(2 * n, dtype=torch.complex128, device="cuda")[::2],
        "host": torch.from_numpy(b),
    }
    for name, t in bad.items():
        for call in (lambda: sgn.wilson_apply(lat, MU, t, out, sgn.F64),
                     lambda: sgn.sign_lanczos_2sided(lat, MU, t, out, k=10),
                     lambda: sgn.multishift_bicgstab(sgn.Problem(lat, MU, t, out), rf),
                     lambda: sgn.sign_arnoldi_rational(lat, MU, good, t, rf, kmax=10),
                     lambda: sgn.sgn_accuracy_measure(lat, good, t)):
            with pytest.raises(sgn.SgnError) as e:
                call()
            assert e.value.status == 1, (name, e.value)
    # canonical FP32 fields are complex64; complex128 ones are refused
    with pytest.raises(sgn.SgnError):
        sgn.wilson_apply(lat, MU, good, out, sgn.F32)
    # per-shift outputs must match the pole count
    with pytest.raises(sgn.SgnError) as e:
        sgn.multishift_solve(sgn.Problem(lat, MU, good, out, x_shift=[torch.empty_like(good)] * 3), rf)
    assert "poles" in str(e.value)
    # a deflation set sized for another lattice
    _, _, L, R, lam = _setup(2)
    big = sgn.Deflation(dev(np.zeros((2, 2 * n), complex)), dev(np.zeros((2, 2 * n), complex)), lam)
    with pytest.raises(sgn.SgnError):
        sgn.sign_lanczos_2sided(lat, MU, good, out, defl=big, k=10)
    # nothing above reached the library: a good call still works and matches the oracle
    sgn.wilson_apply(lat, MU, good, out, sgn.F64)
    ref = WilsonRef(U, DIMS, 0.2).apply(b, MU)
    assert np.linalg.norm(host(out).ravel() - ref) < 1e-13 * np.linalg.norm(ref)
