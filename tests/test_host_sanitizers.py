"""The library's host-only code (small sign, small eigensolver, rational coefficients) and the
oracle's C operator, built with g++/gcc under AddressSanitizer and UndefinedBehaviorSanitizer and
driven over edge and ordinary sizes by tests/host/sanitize_driver.cpp.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0910_1048_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
@pytest.mark.skipif(bool(os.environ.get("LD_PRELOAD")), reason="the sanitizer runtime must be loaded first")
def test_host_code_under_sanitizers(tmp_path):
    out = str(tmp_path)
    oracle_o = os.path.join(out, "wilson_ref.o")
    subprocess.run(["gcc", "-std=c11", *SAN, "-c", os.path.join(ROOT, "oracle", "wilson_ref.c"), "-o", oracle_o],
                   check=True, capture_output=True, text=True)
    exe = os.path.join(out, "sanitize_driver")
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp"),
           os.path.join(CSRC, "small_sign.cpp"), os.path.join(CSRC, "rational.cpp"), oracle_o, "-o", exe, "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "0 failures" in r.stdout
