"""The direct two-sided Lanczos method, restarted FOM-LR and GMRES-LR at the benchmark's
24^3 x 48 size, checked through properties that hold at any size:

  * the direct method computes sign(H_W) b itself: sign(H)^2 = I (the paper's accuracy
    measure) and sign(H) H = H sign(H), the latter with the oracle's operator on the CPU;
  * FOM-LR and GMRES-LR compute the same rational function as the multishift solver, so
    they must agree with an FP64 multishift solve at a tight tolerance, whose every shifted
    system is checked with the oracle's operator on the CPU (the reference is anchored on the
    oracle, not on the library)."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, rational

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

DIMS = (24, 24, 24, 48)
MU = 0.2


def _rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def setup():
    U = synth.gauge_field(DIMS, 0.4, 0)
    b = synth.gaussian_source(DIMS, 0).ravel()
    return U, b, lattice(U, DIMS)


def test_direct_lanczos_full_size_is_a_sign(setup):
    U, b, lat = setup
    kw = dict(k=1000, tol=1e-10, check_every=100)
    bd = dev(b)
    x = torch.empty_like(bd)
    st = sgn.sign_lanczos_2sided(lat, MU, bd, x, **kw)
    ssb = torch.empty_like(bd)
    sgn.sign_lanczos_2sided(lat, MU, x, ssb, **kw)
    acc = sgn.sgn_accuracy_measure(lat, bd, ssb)
    W = WilsonRef(U, DIMS, 0.2)
    hb = W.apply(b, MU).ravel()
    shb = torch.empty_like(bd)
    sgn.sign_lanczos_2sided(lat, MU, dev(hb), shb, **kw)
    hsb = W.apply(host(x), MU).ravel()
    comm = _rel(host(shb), hsb)
    print(f"24^3x48 direct Lanczos: k = {st['iterations']}, accuracy measure {acc:.2e}, "
          f"|S H b - H S b| / |H S b| = {comm:.2e}", flush=True)
    assert acc < 1e-10
    assert comm < 1e-9


@pytest.fixture(scope="module")
def anchored_reference(setup):
    """g_16(cH) b from the FP64 multishift solve to 1e-12 with every shifted solution returned;
    each shifted system's residual y - (c^2 H^2 - sigma_i) x_i is recomputed with the oracle's
    operator, and x = sum_i omega_i x_i is formed on the host."""
    U, b, lat = setup
    rf = sgn.sgn_rational_neuberger(16, 0.12, 2.6)
    om, sg, c = rational.coefficients(16, 0.12, 2.6)
    bd = dev(b)
    xt = torch.empty_like(bd)
    xst = [torch.empty_like(bd) for _ in range(rf.s)]
    sgn.multishift_solve(sgn.Problem(lat, MU, bd, xt, None, xst), rf, tol=1e-12)
    xs = [host(t).ravel() for t in xst]
    del xst
    W = WilsonRef(U, DIMS, 0.2)
    y = c * W.apply(b, MU).ravel()
    ny = np.linalg.norm(y)
    res = [np.linalg.norm(y - (c * c * W.apply(W.apply(xi, MU), MU).ravel() - q * xi)) / ny
           for xi, q in zip(xs, sg)]
    print(f"anchored reference: oracle residuals of the 16 shifted systems {min(res):.1e} .. {max(res):.1e}",
          flush=True)
    assert max(res) < 1e-10
    return rf, om @ np.stack(xs)


@pytest.mark.parametrize("solver", ["fom", "gmres"])
def test_restarted_rational_full_size_matches_anchored_reference(setup, anchored_reference, solver):
    _, b, lat = setup
    rf, xr = anchored_reference
    bd = dev(b)
    f = sgn.sign_arnoldi_rational if solver == "fom" else sgn.sign_gmres_rational
    x = torch.empty_like(bd)
    st = f(lat, MU, bd, x, rf, kmax=30, tol=1e-11)
    e64 = _rel(host(x), xr)
    xm = torch.empty_like(bd)
    stm = f(lat, MU, bd, xm, rf, kmax=30, tol=1e-10, prec=sgn.F32_H16, theta32=1e-2, theta16=1e-5)
    em = _rel(host(xm), xr)
    print(f"24^3x48 {solver}: FP64 {st['restarts']} cycles, vs anchored reference {e64:.2e}; mixed "
          f"{stm['restarts']} cycles, {em:.2e}", flush=True)
    assert e64 < 1e-10
    assert em < 1e-8
