"""Thin ctypes binding of libsgn (argument marshalling only).

Every computation runs inside libsgn.so (HIP kernels for gfx950 and the host
solver code around them).  torch tensors are used only to own device memory
and to provide the stream.  If the library is missing this module raises at
import; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SGN_LIBRARY") or os.path.join(_HERE, "libsgn.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sgn.h")

F64, F32, F32_H16 = 0, 1, 2
NO_GAMMA5, INTERNAL_LAYOUT = 1, 2
LINKS_FULL = 0x100
LINKS_TEMPORAL_GAUGE = 0x200

STATUS = {0: "SGN_OK", 1: "SGN_ERR_INVALID", 2: "SGN_ERR_HIP", 3: "SGN_ERR_NOMEM",
          4: "SGN_ERR_BREAKDOWN", 5: "SGN_ERR_NOT_CONVERGED", 6: "SGN_ERR_IMAG_AXIS",
          7: "SGN_ERR_UNSUPPORTED"}


class SgnError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {detail}")


class LatticeDesc(C.Structure):
    _fields_ = [("dims", C.c_int * 4), ("bc", C.c_int * 4), ("kappa", C.c_double)]


# torch ships its own libamdhip64 and loads it by file name, so a library that
# brought in the system copy first would leave two HIP runtimes in the process
# and the second finds no device.  Importing torch first makes libsgn bind to
# the runtime torch already holds (same soname).
try:
    import torch  # noqa: F401
except ImportError:
    pass

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python paper_0910_1048_amd/build.py`")

lib = C.CDLL(LIB_PATH)
_vp, _i64 = C.c_void_p, C.c_int64
lib.sgn_init.argtypes = [C.POINTER(_vp), C.c_int]
lib.sgn_finalize.argtypes = [_vp]
lib.sgn_status_string.argtypes = [C.c_int]
lib.sgn_status_string.restype = C.c_char_p
lib.sgn_last_error.restype = C.c_char_p
lib.sgn_lattice_create.argtypes = [_vp, C.POINTER(LatticeDesc), _vp, C.c_uint, _vp, C.POINTER(_vp)]
lib.sgn_lattice_destroy.argtypes = [_vp]
lib.sgn_lattice_volume.argtypes = [_vp]
lib.sgn_lattice_link_elements.argtypes = [_vp]
lib.sgn_lattice_volume.restype = _i64
lib.sgn_spinor_bytes.argtypes = [_vp, C.c_int]
lib.sgn_spinor_bytes.restype = C.c_size_t
for _f in ("sgn_spinor_pack", "sgn_spinor_unpack"):
    getattr(lib, _f).argtypes = [_vp, _vp, _vp, C.c_int, _vp]
for _f in ("wilson_apply", "wilson_apply_dag", "wilson_apply_noalloc"):
    getattr(lib, _f).argtypes = [_vp, C.c_double, _vp, _vp, C.c_int, C.c_uint, _vp]


def exported_symbols():
    """Function names declared in include/sgn.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt)) - {"if", "sizeof", "defined"})


def check(status, where):
    if status != 0:
        raise SgnError(status, where, lib.sgn_last_error().decode())


def _invalid(where, detail):
    return SgnError(1, where, detail)


def _tensor(t, where, dtype=None, numel=None, nbytes=None, device=None):
    """Device pointer of t after checking what the C side relies on: a contiguous GPU tensor of
    the expected dtype and size (on the context's device).  Raises SgnError(SGN_ERR_INVALID)
    before anything reaches the library."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise _invalid(where, f"expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise _invalid(where, "tensor is not in GPU memory")
    if device is not None and t.device.index != device:
        raise _invalid(where, f"tensor on device {t.device.index}, the context is on device {device}")
    if dtype is not None and t.dtype != dtype:
        raise _invalid(where, f"dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise _invalid(where, "tensor is not contiguous")
    if numel is not None and t.numel() != numel:
        raise _invalid(where, f"{t.numel()} elements, expected {numel}")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise _invalid(where, f"{t.numel() * t.element_size()} bytes, at least {nbytes} needed")
    return C.c_void_p(t.data_ptr())


def _c128():
    import torch
    return torch.complex128


def _canon_dtype(prec):
    import torch
    return torch.complex128 if int(prec) == F64 else torch.complex64


def _vec(lat, t, where):
    """canonical complex128 vector of the lattice (12 V entries)"""
    return _tensor(t, where, _c128(), 12 * lat.V, device=lat.ctx.device)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Context:
    """sgn_init / sgn_finalize."""

    def __init__(self, device: int = 0):
        h = _vp()
        check(lib.sgn_init(C.byref(h), int(device)), "sgn_init")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            check(lib.sgn_finalize(self.h), "sgn_finalize")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lattice:
    """sgn_lattice_create from canonical complex128 links on the device."""

    def __init__(self, ctx: Context, links, dims, kappa=0.2, bc=(1, 1, 1, -1), prec_mask=0, stream=None):
        d = LatticeDesc()
        for i in range(4):
            d.dims[i] = int(dims[i])
            d.bc[i] = int(bc[i])
        d.kappa = float(kappa)
        vol = 1
        for x in dims:
            vol *= int(x)
        pl = _tensor(links, "sgn_lattice_create: links", _c128(), 36 * vol, device=ctx.device)
        h = _vp()
        check(lib.sgn_lattice_create(ctx.h, C.byref(d), pl, C.c_uint(prec_mask), _stream(stream),
                                     C.byref(h)), "sgn_lattice_create")
        self.h = h
        self.ctx = ctx
        self.dims = tuple(int(x) for x in dims)
        self.kappa = float(kappa)
        self.V = int(lib.sgn_lattice_volume(h))
        self.link_elements = int(lib.sgn_lattice_link_elements(h))
        self.temporal_gauge = bool(prec_mask & LINKS_TEMPORAL_GAUGE)

    def spinor_bytes(self, prec):
        return int(lib.sgn_spinor_bytes(self.h, int(prec)))

    def close(self):
        if self.h:
            check(lib.sgn_lattice_destroy(self.h), "sgn_lattice_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _canon(lat, t, prec, where):
    return _tensor(t, where, _canon_dtype(prec), 12 * lat.V, device=lat.ctx.device)


def _internal(lat, t, prec, where):
    return _tensor(t, where, None, nbytes=lat.spinor_bytes(prec), device=lat.ctx.device)


def _field(lat, t, prec, flags, where):
    """a spinor argument of wilson_apply: canonical (complex128 / complex64 by precision) or the
    library's internal layout (SGN_INTERNAL_LAYOUT: any dtype, spinor_bytes(prec) bytes)"""
    if int(flags) & INTERNAL_LAYOUT:
        return _internal(lat, t, prec, where)
    return _canon(lat, t, prec, where)


def sgn_spinor_pack(lat, canon, internal, prec, stream=None):
    pc = _canon(lat, canon, prec, "sgn_spinor_pack: canon")
    pi = _internal(lat, internal, prec, "sgn_spinor_pack: internal")
    check(lib.sgn_spinor_pack(lat.h, pc, pi, int(prec), _stream(stream)), "sgn_spinor_pack")


def sgn_spinor_unpack(lat, internal, canon, prec, stream=None):
    pi = _internal(lat, internal, prec, "sgn_spinor_unpack: internal")
    pc = _canon(lat, canon, prec, "sgn_spinor_unpack: canon")
    check(lib.sgn_spinor_unpack(lat.h, pi, pc, int(prec), _stream(stream)), "sgn_spinor_unpack")


def wilson_apply(lat, mu, x, out, prec=F64, flags=0, stream=None):
    px = _field(lat, x, prec, flags, "wilson_apply: in")
    po = _field(lat, out, prec, flags, "wilson_apply: out")
    check(lib.wilson_apply(lat.h, float(mu), px, po, int(prec), C.c_uint(flags), _stream(stream)), "wilson_apply")


def wilson_apply_noalloc(lat, mu, x, out, prec=F64, flags=0, stream=None):
    """wilson_apply through the library's static staging array (no device allocation)."""
    px = _field(lat, x, prec, flags, "wilson_apply_noalloc: in")
    po = _field(lat, out, prec, flags, "wilson_apply_noalloc: out")
    check(lib.wilson_apply_noalloc(lat.h, float(mu), px, po, int(prec), C.c_uint(flags), _stream(stream)),
          "wilson_apply_noalloc")


def wilson_apply_dag(lat, mu, x, out, prec=F64, flags=0, stream=None):
    px = _field(lat, x, prec, flags, "wilson_apply_dag: in")
    po = _field(lat, out, prec, flags, "wilson_apply_dag: out")
    check(lib.wilson_apply_dag(lat.h, float(mu), px, po, int(prec), C.c_uint(flags), _stream(stream)),
          "wilson_apply_dag")


# ----------------------------------------------------------------------------- solvers
MAX_POLES = 128


class _Deflation(C.Structure):
    _fields_ = [("m", C.c_int), ("L", _vp), ("R", _vp), ("lam", C.POINTER(C.c_double))]


class LanczosOpts(C.Structure):
    _fields_ = [("k", C.c_int), ("prec", C.c_int), ("tol", C.c_double), ("check_every", C.c_int),
                ("two_pass", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("matvecs", C.c_int), ("restarts", C.c_int),
                ("reliable_updates", C.c_int), ("refine_iterations", C.c_int), ("nshift", C.c_int),
                ("shift_residual", C.c_double * MAX_POLES), ("residual", C.c_double),
                ("min_abs_re", C.c_double), ("krylov_ms", C.c_double), ("small_ms", C.c_double),
                ("total_ms", C.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "shift_residual"}
        d["shift_residual"] = list(self.shift_residual[: self.nshift])
        return d


class Deflation:
    """LR deflation set: L, R device tensors of shape (m, n) complex128 (canonical
    vectors back to back), lam host complex eigenvalues (m,)."""

    def __init__(self, L, R, lam):
        import numpy as np
        self.L, self.R = L, R
        self._lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128)).view(np.float64)
        self.m = int(np.asarray(lam).size)
        pl = _tensor(L, "Deflation: L", _c128())
        pr = _tensor(R, "Deflation: R", _c128())
        if L.numel() != R.numel() or (self.m and L.numel() % self.m):
            raise _invalid("Deflation", f"L and R need m = {self.m} vectors each ({L.numel()}, {R.numel()} entries)")
        self.struct = _Deflation(self.m, pl, pr, self._lam.ctypes.data_as(C.POINTER(C.c_double)))

    def check_for(self, lat, where):
        """the set fits the lattice: m vectors of 12 V entries each, on the context's device"""
        _tensor(self.L, where + ": deflation L", _c128(), self.m * 12 * lat.V, device=lat.ctx.device)
        _tensor(self.R, where + ": deflation R", _c128(), self.m * 12 * lat.V, device=lat.ctx.device)


def _defl_ptr(defl, lat=None, where=""):
    if defl is None:
        return None
    if lat is not None:
        defl.check_for(lat, where)
    return C.byref(defl.struct)


lib.sign_lanczos_2sided.argtypes = [_vp, C.c_double, _vp, _vp, _vp, C.POINTER(LanczosOpts),
                                    C.POINTER(Stats), _vp]


def sign_lanczos_2sided(lat, mu, b, x, defl=None, k=200, prec=F64, tol=0.0, check_every=0, two_pass=False,
                        stream=None):
    """x = sign(H_W(mu)) b by the direct two-sided Lanczos-LR method; returns the stats dict."""
    o = LanczosOpts(int(k), int(prec), float(tol), int(check_every), int(bool(two_pass)))
    st = Stats()
    w = "sign_lanczos_2sided"
    pb, px = _vec(lat, b, w + ": b"), _vec(lat, x, w + ": x")
    check(lib.sign_lanczos_2sided(lat.h, float(mu), pb, px, _defl_ptr(defl, lat, w), C.byref(o), C.byref(st),
                                  _stream(stream)), w)
    return st.as_dict()


class Rational(C.Structure):
    _fields_ = [("s", C.c_int), ("c", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("omega", C.c_double * MAX_POLES), ("sigma", C.c_double * MAX_POLES)]


class _Problem(C.Structure):
    _fields_ = [("lat", _vp), ("mu", C.c_double), ("b", _vp), ("x", _vp), ("defl", C.POINTER(_Deflation)),
                ("x_shift", C.POINTER(_vp))]


class MsOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("prec", C.c_int), ("theta32", C.c_double),
                ("theta16", C.c_double), ("delta", C.c_double), ("poll", C.c_int), ("verify", C.c_int),
                ("basis_slots", C.c_int), ("graph", C.c_int)]


lib.sgn_rational_neuberger.argtypes = [C.c_int, C.c_double, C.c_double, C.POINTER(Rational)]
lib.sgn_poles_needed.argtypes = [C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int)]
lib.multishift_solve.argtypes = [C.POINTER(_Problem), C.c_int, C.POINTER(Rational), C.POINTER(MsOpts),
                                 C.POINTER(Stats), _vp]


def sgn_rational_neuberger(s, alpha, beta):
    r = Rational()
    check(lib.sgn_rational_neuberger(int(s), float(alpha), float(beta), C.byref(r)), "sgn_rational_neuberger")
    return r


def sgn_poles_needed(alpha, beta, eps):
    s = C.c_int()
    check(lib.sgn_poles_needed(float(alpha), float(beta), float(eps), C.byref(s)), "sgn_poles_needed")
    return s.value


lib.sgn_rational_neuberger_rescaled.argtypes = [C.c_int, C.c_double, C.c_double, C.POINTER(Rational),
                                                C.POINTER(C.c_double)]
lib.sgn_rational_zolotarev.argtypes = [C.c_int, C.c_double, C.c_double, C.POINTER(Rational), C.POINTER(C.c_double)]


def sgn_rational_neuberger_rescaled(s, alpha, beta):
    """(coefficients, largest real-axis error on [alpha, beta])."""
    r, e = Rational(), C.c_double()
    check(lib.sgn_rational_neuberger_rescaled(int(s), float(alpha), float(beta), C.byref(r), C.byref(e)),
          "sgn_rational_neuberger_rescaled")
    return r, e.value


def sgn_rational_zolotarev(s, alpha, beta):
    """(coefficients, uniform error on [-beta,-alpha] u [alpha,beta])."""
    r, e = Rational(), C.c_double()
    check(lib.sgn_rational_zolotarev(int(s), float(alpha), float(beta), C.byref(r), C.byref(e)),
          "sgn_rational_zolotarev")
    return r, e.value


lib.sgn_small_sign.argtypes = [C.c_int, _vp, _vp, _vp, _vp, C.POINTER(C.c_double)]


def sgn_small_sign(diag, sub, sup):
    """sign(T) e_1 for the complex tridiagonal T (host); returns (y, min |Re lambda|)."""
    import numpy as np
    d = np.ascontiguousarray(diag, dtype=np.complex128)
    k = d.size
    lo = np.ascontiguousarray(sub, dtype=np.complex128) if k > 1 else None
    up = np.ascontiguousarray(sup, dtype=np.complex128) if k > 1 else None
    if k > 1 and (lo.size != k - 1 or up.size != k - 1):
        raise ValueError("sub and sup need k - 1 entries")
    y = np.empty(k, dtype=np.complex128)
    mr = C.c_double()
    ptr = lambda a: C.c_void_p(a.ctypes.data) if a is not None else None
    check(lib.sgn_small_sign(k, ptr(d), ptr(lo), ptr(up), ptr(y), C.byref(mr)), "sgn_small_sign")
    return y, mr.value


class Problem:
    """One right-hand side of multishift_solve.  x_shift: optional list of s device tensors."""

    def __init__(self, lat, mu, b, x, defl=None, x_shift=None):
        self.lat, self.mu, self.b, self.x, self.defl, self.x_shift = lat, mu, b, x, defl, x_shift


def _problem_array(problems, rational, where):
    """(problem list, ctypes sgn_problem array, objects that must outlive the call), every tensor
    checked against its lattice and every x_shift list against the pole count"""
    if isinstance(problems, Problem):
        problems = [problems]
    n = len(problems)
    arr = (_Problem * max(n, 1))()
    keep = []
    for i, p in enumerate(problems):
        w = f"{where}: problem {i}"
        if p.x_shift is not None and len(p.x_shift) != int(rational.s):
            raise _invalid(w, f"x_shift holds {len(p.x_shift)} vectors, the rational function has "
                              f"{int(rational.s)} poles")
        arr[i].lat = p.lat.h
        arr[i].mu = float(p.mu)
        arr[i].b = _vec(p.lat, p.b, w + " b")
        arr[i].x = _vec(p.lat, p.x, w + " x")
        if p.defl is not None:
            p.defl.check_for(p.lat, w)
            arr[i].defl = C.pointer(p.defl.struct)
        if p.x_shift is not None:
            xs = (_vp * len(p.x_shift))(*[_vec(p.lat, t, f"{w} x_shift[{j}]") for j, t in enumerate(p.x_shift)])
            keep.append(xs)
            arr[i].x_shift = C.cast(xs, C.POINTER(_vp))
    return problems, arr, keep


def multishift_solve(problems, rational, tol=1e-10, maxiter=10000, prec=F64, theta32=0.0, theta16=0.0,
                     delta=0.0, poll=0, verify=False, basis_slots=0, graph=True, stream=None):
    """Multishift BiCG-LR for every problem; returns one stats dict per problem."""
    problems, arr, keep = _problem_array(problems, rational, "multishift_solve")
    n = len(problems)
    o = MsOpts(float(tol), int(maxiter), int(prec), float(theta32), float(theta16), float(delta), int(poll),
               int(bool(verify)), int(basis_slots), 0 if graph else -1)
    st = (Stats * max(n, 1))()
    check(lib.multishift_solve(arr, n, C.byref(rational), C.byref(o), st, _stream(stream)), "multishift_solve")
    return [st[i].as_dict() for i in range(n)]


lib.multishift_bicgstab.argtypes = lib.multishift_solve.argtypes


def multishift_bicgstab(problems, rational, tol=1e-10, maxiter=10000, prec=F64, theta32=0.0, theta16=0.0,
                        delta=0.0, poll=0, basis_slots=0, graph=True, verify=False, stream=None):
    """Multishift BiCGStab for every problem (stored basis and the mixed schedule; basis_slots < 0:
    per-shift vectors, FP64 only); verify: FP64 true residual of every shifted system and FP64
    refinement of those above tol (stored basis).  One stats dict per problem."""
    problems, arr, keep = _problem_array(problems, rational, "multishift_bicgstab")
    n = len(problems)
    o = MsOpts(float(tol), int(maxiter), int(prec), float(theta32), float(theta16), float(delta), int(poll),
               int(bool(verify)), int(basis_slots), 0 if graph else -1)
    st = (Stats * max(n, 1))()
    check(lib.multishift_bicgstab(arr, n, C.byref(rational), C.byref(o), st, _stream(stream)), "multishift_bicgstab")
    return [st[i].as_dict() for i in range(n)]


lib.multishift_qmr.argtypes = lib.multishift_solve.argtypes


def multishift_qmr(problems, rational, tol=1e-10, maxiter=10000, prec=F64, theta32=0.0, theta16=0.0, poll=0,
                   basis_slots=0, verify=False, stream=None):
    """Multishift QMR for every problem (stored Lanczos basis, per-shift least squares, FP64 or the
    mixed stencil schedule); one stats dict per problem."""
    problems, arr, keep = _problem_array(problems, rational, "multishift_qmr")
    n = len(problems)
    o = MsOpts(float(tol), int(maxiter), int(prec), float(theta32), float(theta16), 0.0, int(poll),
               1 if verify else 0, int(basis_slots), 0)
    st = (Stats * max(n, 1))()
    check(lib.multishift_qmr(arr, n, C.byref(rational), C.byref(o), st, _stream(stream)), "multishift_qmr")
    return [st[i].as_dict() for i in range(n)]


K_STENCIL_F64, K_STENCIL_F32, K_STENCIL_H16, K_SHIFT_UPDATE, K_SEED_UPDATE, K_LIFT, K_COUNT = range(7)
KERNEL_NAMES = ["stencil_f64", "stencil_f32", "stencil_h16", "shift_update", "seed_update", "basis_lift"]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_longlong), ("total_ms", C.c_double), ("bytes", C.c_double), ("flops", C.c_double),
                ("calls", C.c_longlong), ("bytes_stored", C.c_double)]


lib.sgn_profile_enable.argtypes = [_vp, C.c_int]
lib.sgn_profile_read.argtypes = [_vp, C.POINTER(KernelProfile)]


def sgn_profile_enable(ctx, enable=True, every=1):
    """Start (and reset) or stop launch profiling; every > 1 records every N-th launch per class."""
    check(lib.sgn_profile_enable(ctx.h, (max(int(every), 1) if enable else 0)), "sgn_profile_enable")


def sgn_profile_read(ctx):
    """{kernel class name: {launches, total_ms, bytes, flops}} of the launches since enable."""
    arr = (KernelProfile * K_COUNT)()
    check(lib.sgn_profile_read(ctx.h, arr), "sgn_profile_read")
    return {KERNEL_NAMES[i]: {"launches": arr[i].launches, "total_ms": arr[i].total_ms, "bytes": arr[i].bytes,
                              "flops": arr[i].flops, "calls": arr[i].calls, "bytes_stored": arr[i].bytes_stored}
            for i in range(K_COUNT)}


lib.wilson_apply_multi.argtypes = [_vp, C.c_int, C.POINTER(C.c_double), C.POINTER(_vp), C.POINTER(_vp), C.c_int,
                                   C.c_uint, _vp]


def wilson_apply_multi(lat, mus, xs, outs, prec=F64, flags=INTERNAL_LAYOUT, stream=None):
    """outs[i] = H_W(mus[i]) xs[i], right-hand sides sharing link loads (internal layout)."""
    n = len(xs)
    if len(mus) != n or len(outs) != n:
        raise _invalid("wilson_apply_multi", "mus, xs and outs need the same length")
    mu = (C.c_double * n)(*[float(m) for m in mus])
    pin = (_vp * n)(*[_field(lat, t, prec, flags, f"wilson_apply_multi: in[{i}]") for i, t in enumerate(xs)])
    pout = (_vp * n)(*[_field(lat, t, prec, flags, f"wilson_apply_multi: out[{i}]") for i, t in enumerate(outs)])
    check(lib.wilson_apply_multi(lat.h, n, mu, pin, pout, int(prec), C.c_uint(flags), _stream(stream)),
          "wilson_apply_multi")


class TuneCandidate(C.Structure):
    _fields_ = [("block_sites", C.c_int), ("links_in_registers", C.c_int), ("us", C.c_double), ("chosen", C.c_int),
                ("t_slices", C.c_int)]


lib.sgn_autotune.argtypes = [_vp, C.c_int, C.c_int, C.c_int, C.POINTER(TuneCandidate), C.c_int,
                             C.POINTER(C.c_int), _vp]


def sgn_autotune(lat, prec, nrhs=1, reps=20, stream=None):
    """Time the stencil's candidate launch shapes for lat's dimensions, prec and nrhs right-hand sides;
    the fastest is kept by the context.  Returns the candidates as dicts (chosen = 1 for the fastest)."""
    arr = (TuneCandidate * 64)()
    n = C.c_int()
    check(lib.sgn_autotune(lat.h, int(prec), int(nrhs), int(reps), arr, 64, C.byref(n), _stream(stream)),
          "sgn_autotune")
    return [{f: getattr(arr[i], f) for f, _ in TuneCandidate._fields_} for i in range(min(n.value, 64))]


lib.sgn_tune_set.argtypes = [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]


def sgn_tune_set(lat, prec, multi=False, max_sites=0, t_slices=1, links_in_registers=-1):
    """Pin the stencil's launch shape for lattices of lat's dimensions (see sgn_autotune)."""
    check(lib.sgn_tune_set(lat.h, int(prec), int(bool(multi)), int(max_sites), int(t_slices),
                           int(links_in_registers)), "sgn_tune_set")


class ArnoldiOpts(C.Structure):
    _fields_ = [("kmax", C.c_int), ("tol", C.c_double), ("max_restarts", C.c_int), ("prec", C.c_int),
                ("theta32", C.c_double), ("theta16", C.c_double)]


lib.sign_arnoldi_rational.argtypes = [_vp, C.c_double, _vp, _vp, C.POINTER(Rational), C.POINTER(_Deflation),
                                      C.POINTER(ArnoldiOpts), C.POINTER(Stats), _vp]


def sign_arnoldi_rational(lat, mu, b, x, rational, defl=None, kmax=40, tol=1e-10, max_restarts=0, prec=F64,
                          theta32=0.0, theta16=0.0, stream=None):
    """x = x_P + g_s(c H_W)(I-P) b by restarted FOM-LR; returns the stats dict."""
    o = ArnoldiOpts(int(kmax), float(tol), int(max_restarts), int(prec), float(theta32), float(theta16))
    st = Stats()
    w = "sign_arnoldi_rational"
    pb, px = _vec(lat, b, w + ": b"), _vec(lat, x, w + ": x")
    d = _defl_ptr(defl, lat, w)
    check(lib.sign_arnoldi_rational(lat.h, float(mu), pb, px, C.byref(rational), d, C.byref(o),
                                    C.byref(st), _stream(stream)), w)
    return st.as_dict()


lib.sign_gmres_rational.argtypes = lib.sign_arnoldi_rational.argtypes


class EigOpts(C.Structure):
    _fields_ = [("m", C.c_int), ("nev", C.c_int), ("kmax", C.c_int), ("tol", C.c_double),
                ("max_restarts", C.c_int), ("seed", C.c_uint)]


lib.sgn_critical_eigenpairs.argtypes = [_vp, C.c_double, C.POINTER(EigOpts), _vp, _vp, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(Stats), _vp]


def sgn_critical_eigenpairs(lat, mu, m, L, R, nev=0, kmax=0, tol=0.0, max_restarts=0, seed=0, stream=None):
    """Left/right eigenvectors of the m eigenvalues of H_W(mu) closest to the imaginary axis
    into the device tensors L and R (m x 12V complex128 each).  Returns (lambda, alpha, stats)."""
    o = EigOpts(int(m), int(nev), int(kmax), float(tol), int(max_restarts), int(seed))
    lam = (C.c_double * (2 * int(m)))()
    alpha = C.c_double()
    st = Stats()
    w = "sgn_critical_eigenpairs"
    pL = _tensor(L, w + ": L", _c128(), int(m) * 12 * lat.V, device=lat.ctx.device)
    pR = _tensor(R, w + ": R", _c128(), int(m) * 12 * lat.V, device=lat.ctx.device)
    check(lib.sgn_critical_eigenpairs(lat.h, float(mu), C.byref(o), pL, pR, lam, C.byref(alpha),
                                      C.byref(st), _stream(stream)), w)
    lm = [complex(lam[2 * i], lam[2 * i + 1]) for i in range(int(m))]
    return lm, alpha.value, st.as_dict()


def sign_gmres_rational(lat, mu, b, x, rational, defl=None, kmax=40, tol=1e-10, max_restarts=0, prec=F64,
                        theta32=0.0, theta16=0.0, stream=None):
    """x = x_P + g_s(c H_W)(I-P) b by restarted GMRES-LR; returns the stats dict."""
    o = ArnoldiOpts(int(kmax), float(tol), int(max_restarts), int(prec), float(theta32), float(theta16))
    st = Stats()
    w = "sign_gmres_rational"
    pb, px = _vec(lat, b, w + ": b"), _vec(lat, x, w + ": x")
    d = _defl_ptr(defl, lat, w)
    check(lib.sign_gmres_rational(lat.h, float(mu), pb, px, C.byref(rational), d, C.byref(o),
                                  C.byref(st), _stream(stream)), w)
    return st.as_dict()


lib.sgn_accuracy_measure.argtypes = [_vp, _vp, _vp, C.POINTER(C.c_double), _vp]


def sgn_accuracy_measure(lat, b, ssb, stream=None):
    """1/2 ||S(S b) - b|| / ||b|| for ssb = S(S b) computed with one approximate sign S."""
    acc = C.c_double()
    w = "sgn_accuracy_measure"
    pb, ps = _vec(lat, b, w + ": b"), _vec(lat, ssb, w + ": ssb")
    check(lib.sgn_accuracy_measure(lat.h, pb, ps, C.byref(acc), _stream(stream)), w)
    return acc.value
