"""Host-code memory and undefined-behaviour checks: the oracle's direct sums
(oracle/direct.c) and the library's host-only truncation-error calls
(csrc/truncation.cpp) built with AddressSanitizer and UndefinedBehavior
Sanitizer (gcc), driven on tiny grids with valid, boundary and invalid
arguments by tests/sanitize/driver.c.  No GPU; the sanitizers end the run
with an error on any out-of-bounds access, leak or undefined operation."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="needs gcc")
def test_sanitized_host_code(tmp_path):
    csrc = os.path.join(ROOT, "paper_1104_0672_amd", "csrc")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + csrc, "-I" + os.path.join(rocm, "include"),
           "-D__HIP_PLATFORM_AMD__"]
    out = str(tmp_path)
    steps = [
        ["gcc"] + SAN + ["-fopenmp", "-c", os.path.join(ROOT, "oracle", "direct.c"), "-o", out + "/direct.o"],
        ["gcc"] + SAN + ["-c", os.path.join(ROOT, "tests", "sanitize", "driver.c"), "-o", out + "/driver.o"],
        ["g++", "-std=c++17", "-x", "c++"] + SAN + inc + ["-c", os.path.join(csrc, "truncation.cpp"),
                                                          "-o", out + "/trunc.o"],
        ["g++", "-std=c++17", "-x", "c++"] + SAN + inc + ["-c", os.path.join(ROOT, "tests", "sanitize", "stubs.cpp"),
                                                          "-o", out + "/stubs.o"],
        ["g++"] + SAN + ["-fopenmp", out + "/driver.o", out + "/direct.o", out + "/trunc.o", out + "/stubs.o",
                         "-o", out + "/drv", "-lm"],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([out + "/drv"], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all calls clean" in r.stdout
