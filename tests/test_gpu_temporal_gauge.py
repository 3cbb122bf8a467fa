"""Lattices in the temporal gauge (SGN_LINKS_TEMPORAL_GAUGE): the field is stored after a colour
rotation G(x) that makes every time link off the last slice the unit matrix, and the stencil skips
those links.  In the canonical layout every result must still be the oracle's, for the field as
given: the operator in every precision and launch shape, the layout round trip, a mixed solve, and
the byte accounting of the skipped links."""
import numpy as np
import pytest

import synth
from oracle import WilsonRef, krylov, rational

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0910_1048_amd as sgn  # noqa: E402
from gpu_util import ctx, dev, host  # noqa: E402

TOL = {sgn.F64: 1e-13, sgn.F32: 1e-6, sgn.F32_H16: 5e-3}
CDT = {sgn.F64: np.complex128, sgn.F32: np.complex64, sgn.F32_H16: np.complex64}
TG = sgn.LINKS_TEMPORAL_GAUGE


def _rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _lat(U, dims, flags=TG, kappa=0.2, bc=(1, 1, 1, -1)):
    return sgn.Lattice(ctx(), dev(U), dims, kappa, bc, prec_mask=flags)


def _run(lat, mu, b, prec, dag=False):
    x = dev(b.astype(CDT[prec]))
    y = torch.empty_like(x)
    (sgn.wilson_apply_dag if dag else sgn.wilson_apply)(lat, mu, x, y, prec)
    return host(y).astype(np.complex128)


# staged whole-plane blocks, bricks, partial planes, the generic kernel (blocks below a wavefront)
@pytest.mark.parametrize("dims", [(4, 6, 4, 8), (8, 8, 8, 16), (3, 5, 2, 7), (2, 2, 2, 4)])
@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_operator_matches_oracle(dims, prec):
    print(f"case dims={dims} prec={prec}", flush=True)
    U = synth.gauge_field(dims, 0.5, 1)
    b = synth.gaussian_source(dims, 2)
    ref = WilsonRef(U, dims, 0.2)
    lat = _lat(U, dims)
    assert lat.link_elements == 6
    for mu in (0.0, 0.3):
        err = _rel(_run(lat, mu, b, prec), ref.apply(b, mu))
        errd = _rel(_run(lat, mu, b, prec, dag=True), ref.apply_adj(b, mu))
        print(f"  mu={mu}: H err {err:.2e}  H^dag err {errd:.2e}", flush=True)
        assert err < TOL[prec] and errd < TOL[prec]


def test_antiperiodic_and_periodic_time_with_kappa():
    """The last slice's time links carry the whole line's product; the boundary factor stays apart."""
    dims = (4, 4, 4, 6)
    U = synth.gauge_field(dims, 0.5, 4)
    b = synth.gaussian_source(dims, 5)
    for bc, kappa in (((1, 1, 1, 1), 0.15), ((-1, 1, -1, -1), 0.25)):
        ref = WilsonRef(U, dims, kappa, bc=bc)
        assert _rel(_run(_lat(U, dims, kappa=kappa, bc=bc), 0.3, b, sgn.F64), ref.apply(b, 0.3)) < 1e-13


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_layout_round_trip_and_internal_fields(prec):
    """pack applies G and unpack G^H (the round trip is the identity up to rounding); the internal
    field differs from the plain lattice's (it holds G psi); an application on internal fields
    equals the canonical-layout call bit for bit."""
    dims = (4, 6, 4, 8)
    U = synth.gauge_field(dims, 0.5, 0)
    b = synth.gaussian_source(dims, 0).astype(CDT[prec])
    lat, plain = _lat(U, dims), _lat(U, dims, 0)
    x = dev(b)
    xi, xp = (torch.empty(l.spinor_bytes(prec), dtype=torch.uint8, device="cuda") for l in (lat, plain))
    back = torch.empty_like(x)
    sgn.sgn_spinor_pack(lat, x, xi, prec)
    sgn.sgn_spinor_pack(plain, x, xp, prec)
    assert not torch.equal(xi, xp)
    sgn.sgn_spinor_unpack(lat, xi, back, prec)
    assert _rel(host(back), b) < (1e-14 if prec == sgn.F64 else 3e-7)
    yi = torch.empty_like(xi)
    y, y2 = torch.empty_like(x), torch.empty_like(x)
    sgn.wilson_apply(lat, 0.3, xi, yi, prec, sgn.INTERNAL_LAYOUT)
    sgn.sgn_spinor_unpack(lat, yi, y, prec)
    sgn.wilson_apply(lat, 0.3, x, y2, prec)
    assert torch.equal(y, y2)


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_equals_the_plain_lattice(prec):
    dims = (8, 8, 8, 16)
    U = synth.gauge_field(dims, 0.4, 6)
    b = synth.gaussian_source(dims, 7)
    e = _rel(_run(_lat(U, dims), 0.2, b, prec), _run(_lat(U, dims, 0), 0.2, b, prec))
    print(f"prec={prec}: temporal gauge vs plain lattice {e:.2e}", flush=True)
    assert e < (5e-14 if prec == sgn.F64 else 2 * TOL[prec])


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_launch_shapes_are_the_same_operator(prec):
    """Skipping a unit link is exact, so every staged shape (one slice, bricks, several caps), the
    unstaged kernel (which reads the unit links) and, with FP16 links and several right-hand sides,
    the register-link form give bit for bit the same result."""
    dims = (12, 12, 12, 24)
    U = synth.gauge_field(dims, 0.4, 5)
    lat = _lat(U, dims)
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
        sgn.sgn_tune_set(lat, prec, False, -1, 1)  # the unstaged kernel: every link loaded
        ref = apply(1)
        tried = 0
        for cap in (0, 384, 96):
            for T in (1, 2):
                try:
                    sgn.sgn_tune_set(lat, prec, False, cap, T)
                except sgn.SgnError:
                    continue  # no block of this shape fits
                tried += 1
                assert torch.equal(apply(1)[0], ref[0]), (cap, T)
        assert tried >= 4
        sgn.sgn_tune_set(lat, prec, True, 0, 1)
        ref3 = apply(3)
        assert torch.equal(ref3[0], ref[0])
        modes = (0, 1) if prec == sgn.F32_H16 else (-1,)
        for regs in modes:
            for T in (1, 2):
                try:
                    sgn.sgn_tune_set(lat, prec, True, 0, T, regs)
                except sgn.SgnError:
                    continue
                for y0, y1 in zip(ref3, apply(3)):
                    assert torch.equal(y0, y1), (regs, T)
        for b, mu, y in zip(srcs, mus, ref3):
            out = torch.empty(b.size, dtype=torch.complex128 if prec == sgn.F64 else torch.complex64, device="cuda")
            sgn.sgn_spinor_unpack(lat, y, out, prec)
            assert _rel(host(out), W.apply(b, mu)) < TOL[prec]
    finally:
        sgn.sgn_tune_set(lat, prec, False, 0, 1)
        sgn.sgn_tune_set(lat, prec, True, 0, 1)


@pytest.mark.parametrize("prec", [sgn.F64, sgn.F32, sgn.F32_H16])
def test_full_size_sampled_sites(prec):
    """24^3 x 48: the oracle at sampled sites, among them every kind of boundary site (the last
    time slice holds the only non-unit time links), with a per-site bound."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0)
    got = _run(_lat(U, dims), 0.2, b, prec).reshape(-1, 4, 3)
    V = 24 ** 3 * 48
    rng = np.random.default_rng(8)
    last = 24 ** 3 * 47 + rng.integers(0, 24 ** 3, 200)
    first = rng.integers(0, 24 ** 3, 200)
    sites = np.unique(np.concatenate([rng.integers(0, V, 2000), first, last, [0, V - 1, 24 ** 3 * 47]]))
    want = WilsonRef(U, dims, 0.2).apply_sites(b, 0.2, sites)
    err = _rel(got[sites], want)
    ws = np.linalg.norm(want.reshape(len(sites), -1), axis=1)
    es = np.linalg.norm((got[sites] - want.reshape(got[sites].shape)).reshape(len(sites), -1), axis=1)
    site_rel = float(np.max(es / ws))
    print(f"24^3x48 temporal gauge prec={prec}: sampled err {err:.2e}, worst site {site_rel:.2e}", flush=True)
    assert err < TOL[prec] and site_rel < 10 * TOL[prec]


def test_mixed_bicgstab_against_oracle():
    dims = (8, 8, 8, 8)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    W = WilsonRef(U, dims, 0.2)
    om, sg, c = rational.coefficients(16, 0.15, 2.6)
    rf = sgn.sgn_rational_neuberger(16, 0.15, 2.6)
    bd = dev(b)
    x = torch.empty_like(bd)
    st = sgn.multishift_bicgstab(sgn.Problem(_lat(U, dims), 0.2, bd, x), rf, tol=1e-10, prec=sgn.F32_H16)[0]
    xo = krylov.multishift_bicgstab(lambda v: W.apply(v, 0.2), b, om, sg, c, tol=1e-11)
    e = _rel(host(x), xo)
    print(f"8^4 mixed BiCGStab, temporal gauge: vs oracle {e:.2e}, {st['iterations']} iterations", flush=True)
    assert e < 1e-8


@pytest.mark.parametrize("prec,name,spinor,link", [(sgn.F64, "stencil_f64", 192, 144),
                                                   (sgn.F32, "stencil_f32", 96, 72),
                                                   (sgn.F32_H16, "stencil_h16", 96, 36)])
def test_stored_bytes_count_the_last_slice_only(prec, name, spinor, link):
    dims = (12, 12, 12, 24)
    lat = _lat(synth.gauge_field(dims, 0.4, 1), dims)
    xi = torch.zeros(lat.spinor_bytes(prec), dtype=torch.uint8, device="cuda")
    yi = torch.empty_like(xi)
    sgn.wilson_apply(lat, 0.2, xi, yi, prec, sgn.INTERNAL_LAYOUT)
    n = 4
    sgn.sgn_profile_enable(ctx(), True, every=1)
    try:
        for _ in range(n):
            sgn.wilson_apply(lat, 0.2, xi, yi, prec, sgn.INTERNAL_LAYOUT)
        torch.cuda.synchronize()
        p = sgn.sgn_profile_read(ctx())[name]
    finally:
        sgn.sgn_profile_enable(ctx(), False)
    V = lat.V
    assert p["launches"] == n
    assert p["bytes"] == pytest.approx(n * (2 * spinor + 4 * link) * V)
    assert p["bytes_stored"] == pytest.approx(n * (2 * spinor + (3 + 1 / 24) * link * 6 / 9) * V)


def test_refused_for_links_outside_su3():
    dims = (4, 4, 4, 6)
    rng = np.random.default_rng(11)
    U = (rng.standard_normal(dims + (4, 3, 3)) + 1j * rng.standard_normal(dims + (4, 3, 3))) * 0.4
    with pytest.raises(sgn.SgnError) as e:
        _lat(U, dims)
    assert e.value.status == 1


def test_full_size_headline_configuration_residuals_with_oracle_operator():
    """24^3 x 48 in the temporal gauge with the mixed schedule of the benchmark (FP64 first chunk,
    then FP32, FP16 links below 1e-6 ||y||, reliable update at a 0.05 drop), tolerance 1e-9: with
    verify every shifted solution is checked in FP64; all 16 satisfy their systems with the oracle's
    operator on the field as given; x is their omega-weighted sum and the unverified result agrees."""
    dims = (24, 24, 24, 48)
    U = synth.gauge_field(dims, 0.4, 0)
    b = synth.gaussian_source(dims, 0).ravel()
    alpha, beta = 0.12, 2.6
    rf = sgn.sgn_rational_neuberger(16, alpha, beta)
    om, sg, c = rational.coefficients(16, alpha, beta)
    lat = _lat(U, dims)
    kw = dict(tol=1e-9, prec=sgn.F32_H16, theta32=1.0, theta16=1e-6, delta=0.05)
    bd = dev(b)
    x_bench = torch.empty_like(bd)
    sgn.multishift_bicgstab(sgn.Problem(lat, 0.2, bd, x_bench), rf, **kw)
    x = torch.empty_like(bd)
    xs = [torch.empty_like(bd) for _ in range(rf.s)]
    st = sgn.multishift_bicgstab(sgn.Problem(lat, 0.2, bd, x, None, xs), rf, verify=True, **kw)[0]
    print(f"24^3x48 temporal gauge, mixed: {st['iterations']} iterations, {st['reliable_updates']} reliable updates, "
          f"refine iterations {st['refine_iterations']}", flush=True)
    W = WilsonRef(U, dims, 0.2)
    y = c * W.apply(b, 0.2).ravel()
    xs = [host(t).ravel() for t in xs]
    for i in range(rf.s):
        Ax = W.apply(W.apply(xs[i], 0.2), 0.2).ravel()
        res = np.linalg.norm(y - (c * c * Ax - sg[i] * xs[i])) / np.linalg.norm(y)
        print(f"  shift {i}: oracle residual {res:.2e}", flush=True)
        assert res < 1.5e-9
    xv = host(x).ravel()
    assert _rel(xv, om @ np.stack(xs)) < 1e-12
    assert _rel(host(x_bench), xv) < 5e-9


def test_lockstep_batch_mixing_gauges_against_oracle():
    """One lockstep BiCGStab batch over temporal-gauge lattices (8^4 with two problems, so a
    multi-RHS stencil group, and 12^4) and a plain 8^4 lattice: the batched stencil launches carry
    each lattice's own flag and every result is unpacked with its own lattice's rotation.  Every
    shifted system verified in FP64; the 8^4 problems against the oracle's multishift BiCGStab."""
    alpha, beta = 0.1, 2.6
    rf = sgn.sgn_rational_neuberger(16, alpha, beta)
    om, sg, c = rational.coefficients(16, alpha, beta)
    d8, d12 = (8, 8, 8, 8), (12, 12, 12, 12)
    U8, U12, V8 = synth.gauge_field(d8, 0.4, 2), synth.gauge_field(d12, 0.4, 3), synth.gauge_field(d8, 0.4, 4)
    lat8, lat12, plain8 = _lat(U8, d8), _lat(U12, d12), _lat(V8, d8, 0)
    cases = [(lat8, U8, d8, 0.2, 11), (lat8, U8, d8, -0.1, 12), (lat12, U12, d12, 0.2, 13), (plain8, V8, d8, 0.3, 14)]
    probs, outs, srcs = [], [], []
    for lat, _, dims, mu, seed in cases:
        b = synth.gaussian_source(dims, seed).ravel()
        bd = dev(b)
        x = torch.empty_like(bd)
        probs.append(sgn.Problem(lat, mu, bd, x))
        outs.append(x)
        srcs.append(b)
    st = sgn.multishift_bicgstab(probs, rf, tol=1e-10, prec=sgn.F32_H16, theta32=1e-2, theta16=1e-5, delta=0.05,
                                 verify=True)
    print(f"mixed-gauge batch: iterations {[s['iterations'] for s in st]}, verified residuals <= "
          f"{max(s['residual'] for s in st):.1e}", flush=True)
    assert max(s["residual"] for s in st) <= 1e-10
    for k, (lat, U, dims, mu, _) in enumerate(cases):
        if dims != d8:
            continue
        W = WilsonRef(U, dims, 0.2)
        ref = krylov.multishift_bicgstab(lambda v: W.apply(v, mu), srcs[k], om, sg, c, tol=1e-11)
        e = _rel(host(outs[k]), ref)
        print(f"  problem {k} (temporal gauge {lat.temporal_gauge}): vs oracle {e:.2e}", flush=True)
        assert e < 1e-9


def test_every_solver_on_the_c1_lattice_against_dense_references():
    """4^4 (eps 0.5, seed 0, kappa 0.2, mu 0.3) stored in the temporal gauge: the direct two-sided
    Lanczos against the dense sign(H) b, restarted FOM-LR and GMRES-LR and the three multishift
    solvers against the dense 16-pole g(cH) b, and the critical eigenpairs with the deflated sign
    against the stored dense eigenvalues, projections and sign (all written by the oracle)."""
    import os
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    g = np.load(os.path.join(gold, "c1_dense.npz"))
    d = np.load(os.path.join(gold, "c1_deflation.npz"))
    dims, mu = (4, 4, 4, 4), 0.3
    lat = _lat(synth.gauge_field(dims, 0.5, 0), dims)
    b = synth.gaussian_source(dims, 0).ravel()
    bd = dev(b)
    x = torch.empty_like(bd)
    sgn.sign_lanczos_2sided(lat, mu, bd, x, k=320)
    e = _rel(host(x), g["sign_b"])
    print(f"C1 temporal gauge: direct Lanczos k=320 vs dense sign {e:.1e}", flush=True)
    assert e < 1e-8
    rf = sgn.sgn_rational_neuberger(16, float(g["alpha"]), float(g["beta"]))
    for fn in (sgn.sign_arnoldi_rational, sgn.sign_gmres_rational):
        fn(lat, mu, bd, x, rf, kmax=30, tol=1e-11)
        e = _rel(host(x), g["g16_b"])
        print(f"  {fn.__name__}: vs dense g16 {e:.1e}", flush=True)
        assert e < 1e-8
    for fn in (sgn.multishift_solve, sgn.multishift_bicgstab, sgn.multishift_qmr):
        fn(sgn.Problem(lat, mu, bd, x), rf, tol=1e-11)
        e = _rel(host(x), g["g16_b"])
        print(f"  {fn.__name__}: vs dense g16 {e:.1e}", flush=True)
        assert e < 1e-8
    m = 15
    L = torch.empty((m, 12 * lat.V), dtype=torch.complex128, device="cuda")
    R = torch.empty_like(L)
    lam, alpha, _ = sgn.sgn_critical_eigenpairs(lat, mu, m, L, R, tol=1e-12)
    lam = np.array(lam)
    Lh, Rh = host(L), host(R)
    c = Lh.conj() @ b
    print(f"  eigenpairs: eigenvalue error {np.abs(lam - d['lam']).max():.1e}", flush=True)
    assert np.abs(lam - d["lam"]).max() < 1e-10
    assert np.abs(Lh.conj() @ Rh.T - np.eye(m)).max() < 1e-10
    assert _rel(Rh.T @ c, d["Pb"]) < 1e-9
    assert _rel(Rh.T @ (np.sign(lam.real) * c), d["xP"]) < 1e-9
    s = sgn.sgn_poles_needed(alpha, float(g["beta"]), 1e-11)
    rfd = sgn.sgn_rational_neuberger(s, alpha, float(g["beta"]))
    sgn.multishift_bicgstab(sgn.Problem(lat, mu, bd, x, sgn.Deflation(L, R, lam)), rfd, tol=1e-11)
    e = _rel(host(x), g["sign_b"])
    print(f"  deflated BiCGStab ({s} poles): vs dense sign {e:.1e}", flush=True)
    assert e < 1e-9
