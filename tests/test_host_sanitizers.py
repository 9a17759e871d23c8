"""The library's host-side setup code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds fd_host.cpp, fd_geometry.cpp and a driver (tests/sanitize/host_checks.cpp)
with g++ -fsanitize=address,undefined and runs it: any out-of-bounds access,
use after free, leak or undefined behaviour aborts the run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1712_00403_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_setup_code_is_sanitizer_clean(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-pthread", os.path.join(HERE, "sanitize", "host_checks.cpp"),
           os.path.join(CSRC, "fd_host.cpp"), os.path.join(CSRC, "fd_geometry.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               FD_HOST_THREADS="4")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip() == "ok"
