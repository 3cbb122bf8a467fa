"""The binding refuses arguments the C side could not use safely (host memory,
wrong dtype, wrong size, per-shift lists of the wrong length) before anything is
passed to the library.  CPU only: the refusals fire before any device access, so
a stand-in lattice object is enough."""
import types

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402

V = 2 * 2 * 2 * 4


def _lat():
    return types.SimpleNamespace(h=None, V=V, dims=(2, 2, 2, 4), ctx=types.SimpleNamespace(device=0),
                                 spinor_bytes=lambda prec: 12 * V * (16 if prec == sgn.F64 else 8))


def _host_vec():
    return torch.zeros(12 * V, dtype=torch.complex128)


def _refused(call, needle=None):
    with pytest.raises(sgn.SgnError) as e:
        call()
    assert e.value.status == 1 and e.value.name == "SGN_ERR_INVALID"
    if needle:
        assert needle in str(e.value), str(e.value)


def test_host_tensors_are_refused_everywhere():
    lat, x, y = _lat(), _host_vec(), _host_vec()
    rf = sgn.sgn_rational_neuberger(8, 0.2, 2.6)
    calls = [
        lambda: sgn.wilson_apply(lat, 0.2, x, y),
        lambda: sgn.wilson_apply_dag(lat, 0.2, x, y),
        lambda: sgn.wilson_apply(lat, 0.2, torch.zeros(lat.spinor_bytes(sgn.F64), dtype=torch.uint8), y,
                                 sgn.F64, sgn.INTERNAL_LAYOUT),
        lambda: sgn.sgn_spinor_pack(lat, x, y, sgn.F64),
        lambda: sgn.sgn_spinor_unpack(lat, x, y, sgn.F64),
        lambda: sgn.sign_lanczos_2sided(lat, 0.2, x, y),
        lambda: sgn.sign_arnoldi_rational(lat, 0.2, x, y, rf),
        lambda: sgn.sign_gmres_rational(lat, 0.2, x, y, rf),
        lambda: sgn.multishift_solve(sgn.Problem(lat, 0.2, x, y), rf),
        lambda: sgn.multishift_bicgstab(sgn.Problem(lat, 0.2, x, y), rf),
        lambda: sgn.multishift_qmr(sgn.Problem(lat, 0.2, x, y), rf),
        lambda: sgn.sgn_critical_eigenpairs(lat, 0.2, 1, x, y),
        lambda: sgn.sgn_accuracy_measure(lat, x, y),
        lambda: sgn.wilson_apply_multi(lat, [0.2], [x], [y]),
    ]
    for c in calls:
        _refused(c, "not in GPU memory")


def test_links_and_deflation_sets_are_checked():
    ctx = types.SimpleNamespace(h=None, device=0)
    _refused(lambda: sgn.Lattice(ctx, torch.zeros(V * 36, dtype=torch.complex128), (2, 2, 2, 4)), "GPU")
    _refused(lambda: sgn.Lattice(ctx, np.zeros(V * 36, complex), (2, 2, 2, 4)), "torch tensor")
    L = torch.zeros((2, 12 * V), dtype=torch.complex128)
    _refused(lambda: sgn.Deflation(L, L, np.ones(2)), "GPU")


def test_per_shift_list_must_match_the_poles():
    lat, x, y = _lat(), _host_vec(), _host_vec()
    rf = sgn.sgn_rational_neuberger(8, 0.2, 2.6)
    for solver in (sgn.multishift_solve, sgn.multishift_bicgstab, sgn.multishift_qmr):
        _refused(lambda: solver(sgn.Problem(lat, 0.2, x, y, x_shift=[x] * 7), rf), "8 poles")


def test_multi_rhs_lists_must_agree():
    lat, x = _lat(), _host_vec()
    _refused(lambda: sgn.wilson_apply_multi(lat, [0.2, 0.1], [x], [x]), "same length")
