"""sgn_autotune: the launch shapes it tries are all the same operator (bitwise: only the block
decomposition differs), the fastest is kept by the context and used afterwards by every launch
of that class (single applications, the multi-RHS form and the solvers), and results stay those
of the oracle."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, krylov, rational

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import dev, host, lattice  # noqa: E402

CDT = {sgn.F64: np.complex128, sgn.F32: np.complex64, sgn.F32_H16: np.complex64}
TOL = {sgn.F64: 1e-13, sgn.F32: 1e-6, sgn.F32_H16: 5e-3}


def _rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
@pytest.mark.parametrize("nrhs", [1, 6])
def test_autotune_keeps_the_operator(prec, nrhs):
    dims = (12, 12, 12, 24)
    U = synth.gauge_field(dims, 0.4, 2)
    lat = lattice(U, dims)
    W = WilsonRef(U, dims, 0.2)
    nb = lat.spinor_bytes(prec)
    srcs = [synth.gaussian_source(dims, 30 + i) for i in range(nrhs)]
    mus = [0.2 - 0.05 * i for i in range(nrhs)]
    xi = []
    for b in srcs:
        t = torch.empty(nb, dtype=torch.uint8, device="cuda")
        sgn.sgn_spinor_pack(lat, dev(b.astype(CDT[prec])), t, prec)
        xi.append(t)

    def apply():
        ys = [torch.empty_like(t) for t in xi]
        if nrhs == 1:
            sgn.wilson_apply(lat, mus[0], xi[0], ys[0], prec, sgn.INTERNAL_LAYOUT)
        else:
            sgn.wilson_apply_multi(lat, mus, xi, ys, prec)
        torch.cuda.synchronize()
        return ys

    before = apply()
    cands = sgn.sgn_autotune(lat, prec, nrhs, reps=5)
    chosen = [c for c in cands if c["chosen"]]
    print(f"prec={prec} nrhs={nrhs}: " + ", ".join(
        f"{c['block_sites']}{'r' if c['links_in_registers'] else ''}:{c['us']:.1f}us" for c in cands), flush=True)
    assert len(cands) >= 2 and len(chosen) == 1
    assert chosen[0]["us"] == min(c["us"] for c in cands)
    after = apply()
    for b, mu, y0, y1 in zip(srcs, mus, before, after):
        assert torch.equal(y0, y1)
        out = torch.empty(b.size, dtype=torch.complex128 if prec == sgn.F64 else torch.complex64, device="cuda")
        sgn.sgn_spinor_unpack(lat, y1, out, prec)
        assert _rel(host(out).astype(np.complex128), W.apply(b, mu)) < TOL[prec]


def test_solvers_after_autotune_match_the_oracle():
    """Tune every precision (including the multi-RHS form the batched solver uses), then the
    mixed BiCGStab solve and a batched BiCG solve of two right-hand sides on the same lattice
    equal the oracle's multishift solves."""
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    lat = lattice(U, dims)
    for prec in (sgn.F64, sgn.F32, sgn.F32_H16):
        sgn.sgn_autotune(lat, prec, 1, reps=3)
        sgn.sgn_autotune(lat, prec, 2, reps=3)
    W = WilsonRef(U, dims, 0.2)
    om, sg, c = rational.coefficients(16, 0.15, 2.6)
    rf = sgn.sgn_rational_neuberger(16, 0.15, 2.6)
    bs = [synth.gaussian_source(dims, k).ravel() for k in (0, 1)]
    refs = [krylov.multishift_bicgstab(lambda v: W.apply(v, 0.2), b, om, sg, c, tol=1e-11) for b in bs]
    bd = dev(bs[0])
    x = torch.empty_like(bd)
    sgn.multishift_bicgstab(sgn.Problem(lat, 0.2, bd, x), rf, tol=1e-10, prec=sgn.F32_H16, theta32=1e-2,
                            theta16=1e-5, delta=0.05)
    assert _rel(host(x), refs[0]) < 1e-8
    probs = [sgn.Problem(lat, 0.2, dev(b), torch.empty_like(bd)) for b in bs]
    sgn.multishift_solve(probs, rf, tol=1e-10, prec=sgn.F32_H16, theta32=1e-1, theta16=1e-3, delta=0.05)
    for p, r in zip(probs, refs):
        assert _rel(host(p.x), r) < 1e-8


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
@pytest.mark.parametrize("dims", [(12, 12, 12, 24), (4, 6, 4, 8), (6, 4, 6, 10), (24, 24, 24, 48)])
def test_bricks_are_the_same_operator(prec, dims):
    """Blocks of two t-slices (pinned with sgn_tune_set at several site caps), and for one
    right-hand side the kernel without LDS staging, give bit for bit the result of one-slice
    blocks, for one and for three right-hand sides, and the oracle's operator (every site at the
    small sizes, sampled sites at 24^3 x 48)."""
    U = synth.gauge_field(dims, 0.4, 5)
    lat = lattice(U, dims)
    W = WilsonRef(U, dims, 0.2)
    nb = lat.spinor_bytes(prec)
    srcs = [synth.gaussian_source(dims, 40 + i) for i in range(3)]
    mus = [0.2, -0.1, 0.3]
    xi = []
    for b in srcs:
        t = torch.empty(nb, dtype=torch.uint8, device="cuda")
        sgn.sgn_spinor_pack(lat, dev(b.astype(CDT[prec])), t, prec)
        xi.append(t)

    def apply(nrhs):
        ys = [torch.empty_like(t) for t in xi[:nrhs]]
        if nrhs == 1:
            sgn.wilson_apply(lat, mus[0], xi[0], ys[0], prec, sgn.INTERNAL_LAYOUT)
        else:
            sgn.wilson_apply_multi(lat, mus[:nrhs], xi[:nrhs], ys, prec)
        torch.cuda.synchronize()
        return ys

    try:
        for multi, nrhs in ((False, 1), (True, 3)):
            sgn.sgn_tune_set(lat, prec, multi, 0, 1)
            ref = apply(nrhs)
            tried = 0
            for cap in (0, 384, 192, 96):
                try:
                    sgn.sgn_tune_set(lat, prec, multi, cap, 2)
                except sgn.SgnError:
                    continue  # no brick of this cap fits the lattice
                tried += 1
                got = apply(nrhs)
                for y0, y1 in zip(ref, got):
                    assert torch.equal(y0, y1), f"cap {cap}, nrhs {nrhs}"
            assert tried >= 1
            if not multi:  # the kernel without LDS staging
                sgn.sgn_tune_set(lat, prec, False, -1, 1)
                got = apply(1)
                assert torch.equal(ref[0], got[0]), "unstaged kernel"
            for b, mu, y in zip(srcs, mus, ref):
                out = torch.empty(b.size, dtype=torch.complex128 if prec == sgn.F64 else torch.complex64, device="cuda")
                sgn.sgn_spinor_unpack(lat, y, out, prec)
                got = host(out).astype(np.complex128)
                if lat.V <= 20000:
                    assert _rel(got, W.apply(b, mu)) < TOL[prec]
                else:
                    sites = np.random.default_rng(3).choice(lat.V, 400, replace=False)
                    want = W.apply_sites(b, mu, sites)
                    g = got.reshape(lat.V, 4, 3)[sites]
                    assert np.linalg.norm(g - want) / np.linalg.norm(want) < TOL[prec]
    finally:
        sgn.sgn_tune_set(lat, prec, False, 0, 1)
        sgn.sgn_tune_set(lat, prec, True, 0, 1)


def test_tune_set_refusals():
    dims = (4, 4, 4, 5)
    lat = lattice(synth.gauge_field(dims, 0.4, 0), dims)
    with pytest.raises(sgn.SgnError):
        sgn.sgn_tune_set(lat, sgn.F32, False, 0, 2)   # odd L_t: no brick
    with pytest.raises(sgn.SgnError):
        sgn.sgn_tune_set(lat, sgn.F32, False, 0, 3)
    with pytest.raises(sgn.SgnError):
        sgn.sgn_tune_set(lat, sgn.F32, False, -2, 1)
