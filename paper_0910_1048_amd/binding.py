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
LIB_PATH = os.path.join(_HERE, "libsgn.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sgn.h")

F64, F32, F32_H16 = 0, 1, 2
NO_GAMMA5, INTERNAL_LAYOUT = 1, 2

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


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_0910_1048_amd.build`")

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
lib.sgn_lattice_volume.restype = _i64
lib.sgn_spinor_bytes.argtypes = [_vp, C.c_int]
lib.sgn_spinor_bytes.restype = C.c_size_t
for _f in ("sgn_spinor_pack", "sgn_spinor_unpack"):
    getattr(lib, _f).argtypes = [_vp, _vp, _vp, C.c_int, _vp]
for _f in ("wilson_apply", "wilson_apply_dag"):
    getattr(lib, _f).argtypes = [_vp, C.c_double, _vp, _vp, C.c_int, C.c_uint, _vp]


def exported_symbols():
    """Function names declared in include/sgn.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt)) - {"if", "sizeof", "defined"})


def check(status, where):
    if status != 0:
        raise SgnError(status, where, lib.sgn_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


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
        h = _vp()
        check(lib.sgn_lattice_create(ctx.h, C.byref(d), _ptr(links), C.c_uint(prec_mask), _stream(stream),
                                     C.byref(h)), "sgn_lattice_create")
        self.h = h
        self.ctx = ctx
        self.dims = tuple(int(x) for x in dims)
        self.kappa = float(kappa)
        self.V = int(lib.sgn_lattice_volume(h))

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


def sgn_spinor_pack(lat, canon, internal, prec, stream=None):
    check(lib.sgn_spinor_pack(lat.h, _ptr(canon), _ptr(internal), int(prec), _stream(stream)), "sgn_spinor_pack")


def sgn_spinor_unpack(lat, internal, canon, prec, stream=None):
    check(lib.sgn_spinor_unpack(lat.h, _ptr(internal), _ptr(canon), int(prec), _stream(stream)),
          "sgn_spinor_unpack")


def wilson_apply(lat, mu, x, out, prec=F64, flags=0, stream=None):
    check(lib.wilson_apply(lat.h, float(mu), _ptr(x), _ptr(out), int(prec), C.c_uint(flags), _stream(stream)),
          "wilson_apply")


def wilson_apply_dag(lat, mu, x, out, prec=F64, flags=0, stream=None):
    check(lib.wilson_apply_dag(lat.h, float(mu), _ptr(x), _ptr(out), int(prec), C.c_uint(flags),
                               _stream(stream)), "wilson_apply_dag")
