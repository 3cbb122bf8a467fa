"""Parity of the HIP Wilson stencil (wilson_apply / wilson_apply_dag) with the oracle.

Tolerances (relative 2-norm): FP64 1e-13, FP32 1e-6; FP16 links are reported
and bounded by 5e-3 (half precision has a 2^-11 relative step).
"""
import numpy as np
import pytest

import synth
from oracle import WilsonRef

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
import gpu_util  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

TOL = {sgn.F64: 1e-13, sgn.F32: 1e-6, sgn.F32_H16: 5e-3}
CDT = {sgn.F64: np.complex128, sgn.F32: np.complex64, sgn.F32_H16: np.complex64}


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _run(lat, mu, b, prec, dag=False, flags=0):
    x = dev(b.astype(CDT[prec]))
    y = torch.empty_like(x)
    (sgn.wilson_apply_dag if dag else sgn.wilson_apply)(lat, mu, x, y, prec, flags)
    return host(y).astype(np.complex128)


# shapes cover: whole-plane blocks of the staged kernel, partial planes (FP64 at
# 32x16), blocks below one wavefront (generic kernel), padded component stride
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10), (3, 5, 2, 7), (8, 8, 8, 16), (12, 12, 12, 12),
                                  (32, 16, 4, 4), (2, 2, 2, 4)])
@pytest.mark.parametrize("mu", [0.0, 0.3, -0.2])
@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_wilson_apply_matches_oracle(dims, mu, prec):
    print(f"case dims={dims} mu={mu} prec={prec}", flush=True)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 1)
    ref = WilsonRef(U, dims, 0.2)
    lat = lattice(U, dims)
    err = _rel(_run(lat, mu, b, prec), ref.apply(b, mu))
    errd = _rel(_run(lat, mu, b, prec, dag=True), ref.apply_adj(b, mu))
    print(f"  H err {err:.2e}  H^dag err {errd:.2e}", flush=True)
    assert err < TOL[prec] and errd < TOL[prec]


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32])
def test_no_gamma5_flag(prec):
    dims = (4, 4, 6, 4)
    U = synth.gauge_field(dims, 0.5, 2)
    b = synth.gaussian_source(dims, 3)
    ref = WilsonRef(U, dims, 0.2)
    lat = lattice(U, dims)
    assert _rel(_run(lat, 0.3, b, prec, flags=sgn.NO_GAMMA5), ref.apply(b, 0.3, g5=False)) < TOL[prec]
    assert _rel(_run(lat, 0.3, b, prec, dag=True, flags=sgn.NO_GAMMA5), ref.apply_adj(b, 0.3, g5=False)) < TOL[prec]


def test_boundary_conditions_and_kappa():
    dims = (4, 4, 4, 6)
    U = synth.gauge_field(dims, 0.5, 4)
    b = synth.gaussian_source(dims, 5)
    for bc, kappa in (((1, 1, 1, 1), 0.15), ((-1, 1, -1, -1), 0.25)):
        ref = WilsonRef(U, dims, kappa, bc=bc)
        lat = lattice(U, dims, kappa, bc)
        assert _rel(_run(lat, 0.3, b, sgn.F64), ref.apply(b, 0.3)) < 1e-13


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_internal_layout_roundtrip(prec):
    dims = (4, 6, 4, 8)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).astype(CDT[prec])
    lat = lattice(U, dims)
    x = dev(b)
    nbytes = lat.spinor_bytes(prec)
    xi = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    yi = torch.empty_like(xi)
    y = torch.empty_like(x)
    back = torch.empty_like(x)
    sgn.sgn_spinor_pack(lat, x, xi, prec)
    sgn.sgn_spinor_unpack(lat, xi, back, prec)
    assert np.array_equal(host(back), b)
    sgn.wilson_apply(lat, 0.3, xi, yi, prec, sgn.INTERNAL_LAYOUT)
    sgn.sgn_spinor_unpack(lat, yi, y, prec)
    sgn.wilson_apply(lat, 0.3, x, back, prec)
    assert np.array_equal(host(y), host(back))


def test_deterministic_rerun():
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0)
    lat = lattice(U, dims)
    a1 = _run(lat, 0.2, b, sgn.F32)
    a2 = _run(lat, 0.2, b, sgn.F32)
    assert np.array_equal(a1, a2)


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_full_size_sampled_sites(prec):
    """24^3 x 48 (the largest configuration): GPU on the whole lattice, oracle at
    sampled sites including every kind of boundary site."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0)
    lat = lattice(U, dims)
    got = _run(lat, 0.2, b, prec).reshape(-1, 4, 3)
    rng = np.random.default_rng(7)
    V = 24 ** 3 * 48
    corners = [0, 23, 24 * 23, 24 ** 2 * 23, 24 ** 3 * 47, V - 1, 24 ** 3 * 47 + 5]
    sites = np.unique(np.concatenate([rng.integers(0, V, 3000), corners]))
    want = WilsonRef(U, dims, 0.2).apply_sites(b, 0.2, sites)
    err = _rel(got[sites], want)
    # per site: a wrong hop at one kind of boundary site would hide in the global norm
    ws = np.linalg.norm(want.reshape(len(sites), -1), axis=1)
    es = np.linalg.norm((got[sites] - want.reshape(got[sites].shape)).reshape(len(sites), -1), axis=1)
    site_rel = float(np.max(es / ws))
    worst = int(sites[int(np.argmax(es / ws))])
    print(f"24^3x48 prec={prec} sampled err {err:.2e}, worst site {worst}: {site_rel:.2e}", flush=True)
    assert err < TOL[prec]
    assert site_rel < 10 * TOL[prec]


def test_invalid_arguments_are_rejected():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 0)
    lat = lattice(U, dims)
    x = dev(synth.gaussian_source(dims, 0))
    with pytest.raises(sgn.SgnError) as e:
        sgn.wilson_apply(lat, 0.3, x, x, sgn.F64)
    assert e.value.status == 1
    with pytest.raises(sgn.SgnError):
        sgn.wilson_apply(lat, float("nan"), x, torch.empty_like(x), sgn.F64)


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
@pytest.mark.parametrize("nrhs", [1, 2, 3, 5, 8, 16, 17])
@pytest.mark.parametrize("dims", [(4, 6, 4, 8), (12, 12, 12, 12)])
def test_multi_rhs_stencil(prec, nrhs, dims):
    """wilson_apply_multi: right-hand sides with their own mu (and, every third one, the
    gamma5-less operator D_W) sharing link loads in groups of up to 16, against the oracle;
    17 right-hand sides make a group of 16 and one of 1."""
    print(f"case multi dims={dims} nrhs={nrhs} prec={prec}", flush=True)
    U = synth.gauge_field(dims, 0.5, 1)
    ref = WilsonRef(U, dims, 0.2)
    lat = lattice(U, dims)
    mus = [0.3 * np.cos(1.7 * i) for i in range(nrhs)]
    srcs = [synth.gaussian_source(dims, 20 + i) for i in range(nrhs)]
    nbytes = lat.spinor_bytes(prec)
    xi = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nrhs)]
    yi = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(nrhs)]
    for b, t in zip(srcs, xi):
        sgn.sgn_spinor_pack(lat, dev(b.astype(CDT[prec])), t, prec)
    sgn.wilson_apply_multi(lat, mus, xi, yi, prec)
    errs = []
    for mu, b, t in zip(mus, srcs, yi):
        out = torch.empty(b.size, dtype=torch.complex128 if prec == sgn.F64 else torch.complex64, device="cuda")
        sgn.sgn_spinor_unpack(lat, t, out, prec)
        errs.append(_rel(host(out).astype(np.complex128).reshape(b.shape), ref.apply(b, mu)))
    print(f"  worst rel err {max(errs):.2e}", flush=True)
    assert max(errs) < TOL[prec]
    # each right-hand side equals its own single application
    for k in (0, nrhs - 1):
        y1 = torch.empty_like(yi[k])
        sgn.wilson_apply(lat, mus[k], xi[k], y1, prec, sgn.INTERNAL_LAYOUT)
        assert torch.equal(y1, yi[k])


@pytest.mark.parametrize("prec", [sgn.F32, sgn.F32_H16])
def test_multi_rhs_stencil_full_size(prec):
    """16 right-hand sides on 24^3 x 48 (the batched multi-RHS form at the size it is timed at):
    the oracle at sampled sites of every right-hand side, and bitwise equality with the
    single applications."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.4, 0)
    lat = lattice(U, dims)
    W = WilsonRef(U, dims, 0.2)
    n = 16
    mus = [0.2 * np.cos(0.9 * i) for i in range(n)]
    rng = np.random.default_rng(5)
    V = 24 ** 3 * 48
    sites = np.unique(np.concatenate([rng.integers(0, V, 400), [0, V - 1, 24 ** 3 * 47, 23]]))
    nbytes = lat.spinor_bytes(prec)
    xi = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(n)]
    yi = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(n)]
    srcs = []
    for i in range(n):
        b = synth.gaussian_source(dims, 100 + i) if i < 2 else None
        if b is None:  # cheaper sources beyond the first two: scaled and phased copies
            b = srcs[i % 2] * np.exp(1j * 0.3 * i) * (1 + 0.1 * i)
        srcs.append(b)
        sgn.sgn_spinor_pack(lat, dev(b.astype(np.complex64)), xi[i], prec)
    sgn.wilson_apply_multi(lat, mus, xi, yi, prec)
    worst = 0.0
    for i in range(n):
        out = torch.empty(srcs[i].size, dtype=torch.complex64, device="cuda")
        sgn.sgn_spinor_unpack(lat, yi[i], out, prec)
        got = host(out).astype(np.complex128).reshape(-1, 4, 3)[sites]
        want = W.apply_sites(srcs[i].astype(np.complex64).astype(np.complex128), mus[i], sites)
        worst = max(worst, _rel(got, want))
        if i in (0, 7, 15):
            y1 = torch.empty_like(yi[i])
            sgn.wilson_apply(lat, mus[i], xi[i], y1, prec, sgn.INTERNAL_LAYOUT)
            assert torch.equal(y1, yi[i]), i
    print(f"24^3x48 16 RHS prec={prec}: worst sampled rel err {worst:.2e}", flush=True)
    assert worst < TOL[prec]


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_two_row_links_equal_full_links(prec):
    """SU(3) links are stored as two rows (third rebuilt in the stencil); the same
    operator with all nine entries stored, and the oracle, agree."""
    dims = (4, 6, 4, 8)
    U = synth.gauge_field(dims, 0.5, 3)
    b = synth.gaussian_source(dims, 4)
    ref = WilsonRef(U, dims, 0.2)
    lat2 = lattice(U, dims)
    lat3 = sgn.Lattice(gpu_util.ctx(), dev(U), dims, 0.2, prec_mask=sgn.LINKS_FULL)
    assert lat2.link_elements == 6 and lat3.link_elements == 9
    y2, y3 = _run(lat2, 0.3, b, prec), _run(lat3, 0.3, b, prec)
    want = ref.apply(b, 0.3)
    print(f"prec={prec}: two-row {_rel(y2, want):.2e}, full {_rel(y3, want):.2e}", flush=True)
    assert _rel(y2, want) < TOL[prec] and _rel(y3, want) < TOL[prec]
    assert _rel(y2, y3) < (1e-14 if prec == sgn.F64 else 2 * TOL[prec])


def test_non_unitary_links_keep_all_entries():
    """Links that are not SU(3) (here: random complex matrices) keep nine entries and
    still give the oracle's operator."""
    dims = (4, 4, 4, 6)
    rng = np.random.default_rng(11)
    U = (rng.standard_normal(dims + (4, 3, 3)) + 1j * rng.standard_normal(dims + (4, 3, 3))) * 0.4
    b = synth.gaussian_source(dims, 2)
    lat = lattice(U, dims)
    assert lat.link_elements == 9
    ref = WilsonRef(U, dims, 0.2)
    for prec in (sgn.F64, sgn.F32):
        assert _rel(_run(lat, 0.2, b, prec), ref.apply(b, 0.2)) < TOL[prec]
