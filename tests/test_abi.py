"""The C-ABI library loads and exports every function include/sgn.h declares (no GPU needed)."""
import ctypes
import subprocess

import paper_0910_1048_amd as sgn


def test_header_symbols_exported():
    names = sgn.exported_symbols()
    assert "wilson_apply" in names and "wilson_apply_dag" in names
    for n in names:
        assert hasattr(sgn.lib, n), f"libsgn.so does not export {n}"


def test_no_torch_types_in_abi():
    txt = open(sgn.HEADER).read()
    for bad in ("torch", "at::", "Tensor", "c10"):
        assert bad not in txt


def test_status_strings_without_gpu():
    f = sgn.lib.sgn_status_string
    assert f(0) == b"ok"
    assert f(4) == b"Krylov breakdown"
    assert f(99) == b"unknown status"


def test_library_is_gfx950_code_object():
    out = subprocess.run(["/opt/rocm/llvm/bin/llvm-readelf", "-n", sgn.LIB_PATH], capture_output=True, text=True)
    # the offload bundle inside the host library names the target
    data = open(sgn.LIB_PATH, "rb").read()
    assert b"gfx950" in data
