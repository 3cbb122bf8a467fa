"""The per-kernel launch profile (sgn_profile_enable / sgn_profile_read): launch counts, sampling,
the byte model of the stencil and launch times that the kernels' dispatches stamp themselves."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import ctx, dev, lattice  # noqa: E402


def _profile(fn, every=1):
    sgn.sgn_profile_enable(ctx(), True, every=every)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        return sgn.sgn_profile_read(ctx()), wall_ms
    finally:
        sgn.sgn_profile_enable(ctx(), False)


@pytest.mark.parametrize("prec,name,spinor,link", [(sgn.F64, "stencil_f64", 192, 144),
                                                   (sgn.F32, "stencil_f32", 96, 72),
                                                   (sgn.F32_H16, "stencil_h16", 96, 36)])
def test_stencil_launches_and_byte_model(prec, name, spinor, link):
    """n applications record n launches of their class (and nothing else), with the algorithmic
    bytes of the byte model (two spinors and four nine-entry links per site), the stored bytes of
    the links as kept (two rows of SU(3) links), and positive times below the wall clock."""
    dims = (12, 12, 12, 24)
    lat = lattice(synth.gauge_field(dims, 0.4, 1), dims)
    nb = lat.spinor_bytes(prec)
    xi = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    yi = torch.empty_like(xi)
    sgn.wilson_apply(lat, 0.2, xi, yi, prec, sgn.INTERNAL_LAYOUT)
    n = 12
    prof, wall_ms = _profile(lambda: [sgn.wilson_apply(lat, 0.2, xi, yi, prec, sgn.INTERNAL_LAYOUT) for _ in range(n)])
    p = prof[name]
    assert p["calls"] == n and p["launches"] == n
    assert all(v["calls"] == 0 for k, v in prof.items() if k != name)
    V = lat.V
    assert p["bytes"] == pytest.approx(n * (2 * spinor + 4 * link) * V)
    assert lat.link_elements in (6, 9)  # two-row links for SU(3) fields
    assert p["bytes_stored"] == pytest.approx(n * (2 * spinor + 4 * link * lat.link_elements // 9) * V)
    assert 0 < p["total_ms"] < wall_ms
    print(f"{name}: {p['total_ms'] / n * 1e3:.1f} us per launch (wall {wall_ms / n * 1e3:.1f} us)", flush=True)


def test_sampling_and_solver_classes():
    """every = 3 records one launch in three of each class; a mixed BiCGStab solve reports its
    stencil, vector-update and lift classes, each with positive times and bytes."""
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    lat = lattice(U, dims)
    bd = dev(synth.gaussian_source(dims, 0).ravel())
    x = torch.empty_like(bd)
    rf = sgn.sgn_rational_neuberger(16, 0.15, 2.6)
    kw = dict(tol=1e-9, prec=sgn.F32_H16, theta32=1e-2, theta16=1e-5, delta=0.1)
    sgn.multishift_bicgstab(sgn.Problem(lat, 0.2, bd, x), rf, **kw)
    for every in (1, 3):
        prof, _ = _profile(lambda: sgn.multishift_bicgstab(sgn.Problem(lat, 0.2, bd, x), rf, **kw), every)
        for k in ("stencil_f64", "stencil_f32", "stencil_h16", "shift_update", "seed_update", "basis_lift"):
            p = prof[k]
            assert p["calls"] > 0, k
            assert p["launches"] == (p["calls"] + every - 1) // every, (k, every)
            assert p["total_ms"] > 0 and p["bytes"] > 0, k
        if every == 1:
            calls1 = {k: v["calls"] for k, v in prof.items()}
        else:  # the same solve: the same launches, a third of them timed
            assert {k: v["calls"] for k, v in prof.items()} == calls1
    assert np.isfinite(torch.linalg.norm(x).item())
