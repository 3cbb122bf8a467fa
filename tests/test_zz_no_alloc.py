"""wilson_apply_noalloc: the variant of wilson_apply that allocates nothing (its staging
lives in a static device array) gives the same bits as wilson_apply, on two calls in a
row with the second on a smaller lattice, in every precision; it refuses a lattice whose
fields do not fit the array."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

CDT = {sgn.F64: np.complex128, sgn.F32: np.complex64, sgn.F32_H16: np.complex64}


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_noalloc_equals_wilson_apply(prec):
    # first the largest FP64 lattice the array takes (16^4), then a smaller one
    for dims, mu, seed in (((16, 16, 16, 16), 0.2, 0), ((4, 6, 4, 8), 0.3, 1)):
        U = synth.gauge_field(dims, 0.4, seed)
        b = synth.gaussian_source(dims, seed).ravel().astype(CDT[prec])
        lat = lattice(U, dims)
        x = dev(b)
        y_ref = torch.empty_like(x)
        y = torch.full_like(x, float("nan"))
        sgn.wilson_apply(lat, mu, x, y_ref, prec)
        sgn.wilson_apply_noalloc(lat, mu, x, y, prec)
        yr, yn = host(y_ref), host(y)
        print(f"prec={prec} {dims}: noalloc vs wilson_apply max |diff| {np.abs(yn - yr).max():.1e}", flush=True)
        assert np.array_equal(yn, yr)
        if prec == sgn.F64:
            ref = WilsonRef(U, dims, 0.2).apply(b, mu).ravel()
            assert np.linalg.norm(yn - ref) < 1e-13 * np.linalg.norm(ref)
        # gamma5-less operator and the internal layout go through the same entry point
        sgn.wilson_apply(lat, mu, x, y_ref, prec, sgn.NO_GAMMA5)
        sgn.wilson_apply_noalloc(lat, mu, x, y, prec, sgn.NO_GAMMA5)
        assert np.array_equal(host(y), host(y_ref))


def test_noalloc_refuses_a_lattice_beyond_the_array():
    dims = (16, 16, 16, 32)  # FP64 staging of 2 x 25.3 MB: beyond the 25.3 MB array
    U = synth.gauge_field(dims, 0.4, 0)
    lat = lattice(U, dims)
    x = dev(synth.gaussian_source(dims, 0).ravel())
    with pytest.raises(sgn.SgnError) as e:
        sgn.wilson_apply_noalloc(lat, 0.2, x, torch.empty_like(x), sgn.F64)
    assert e.value.status == 1 and "SGN_NOALLOC_MAX_BYTES" in str(e.value)
    # FP32 fields of the same lattice fit
    x32 = x.to(torch.complex64)
    y32, r32 = torch.empty_like(x32), torch.empty_like(x32)
    sgn.wilson_apply_noalloc(lat, 0.2, x32, y32, sgn.F32)
    sgn.wilson_apply(lat, 0.2, x32, r32, sgn.F32)
    assert np.array_equal(host(y32), host(r32))
