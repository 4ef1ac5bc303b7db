"""The host-only small dense FP64 solvers of libhyeig (csrc/smalldense.cpp:
symmetric and band eigenproblems, Cholesky, triangular inverse, the
Rayleigh-Ritz pencil, DIIS, the 2x2 pencil) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run on the driver
tests/sanitize_smalldense.cpp, which checks each result against its defining
identity.  CPU only: no GPU code is built or run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_smalldense_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_smalldense")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize_smalldense.cpp"),
           os.path.join(ROOT, "paper_2305_15552_amd", "csrc", "smalldense.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok: 0 failure(s)" in r.stdout
