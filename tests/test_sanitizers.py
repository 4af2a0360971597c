"""AddressSanitizer + UndefinedBehaviorSanitizer builds of host code, run on
the CPU: the library's approximant preparation and both Remez exchanges
(approx.cpp, remez.cpp; tests/sanitize/host_driver.cpp) and the FP64 oracle
(oracle.c; tests/sanitize/oracle_driver.c). Any invalid access, leak or
undefined behaviour aborts the driver (-fno-sanitize-recover=all), so the test
asserts a clean exit and a clean stderr. Built with the ROCm host compiler
(its clang has the sanitizer runtimes and _Float16 on x86)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

pytestmark = pytest.mark.skipif(not (os.path.exists(CLANG) and shutil.which("ld")), reason="no host clang")


def build_and_run(cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    for bad in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:"):
        assert bad not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_host_cpp_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_1009_0959_amd", "csrc")
    exe = str(tmp_path / "host_drv")
    out = build_and_run([CLANG + "++", "-std=c++17", *SAN, "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
                         os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                         os.path.join(csrc, "approx.cpp"), os.path.join(csrc, "remez.cpp"), "-o", exe], exe)
    assert "accepted" in out


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "orc_drv")
    out = build_and_run([CLANG, "-std=c11", *SAN, "-ffp-contract=off",
                         os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe], exe)
    assert "1800 configurations" in out
