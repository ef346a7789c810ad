"""The plan's host eigensolver (csrc/eig.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no GPU code) and run over uniform, graded,
stretched and tiny axes, up to the 575-node global axis of the large grid:
no sanitizer report, and the residuals of D W = W Lambda and W^{-1} W = I,
recomputed by the driver from D = M^{-1} K, within bounds (Sec. 2, the 1D
generalized eigenproblems of the block and global axes)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_01299_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_eigensolver_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "eig_check")
        build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", "-I", CSRC, os.path.join(ROOT, "tests", "host", "eig_check.cpp"),
                 os.path.join(CSRC, "eig.cpp"), "-o", exe]
        r = subprocess.run(build, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
        assert "all ok" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
