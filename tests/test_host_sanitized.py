"""The library's host-only C++ (partition.cpp, order.cpp, host.cpp) built
with AddressSanitizer and UndefinedBehaviorSanitizer and run on the checks of
tests/native/host_checks.cpp: partitioners on graphs of 1 to 3000 vertices
(edgeless, sparse, dense; K from 1 to n), reverse Cuthill-McKee orders,
argument validation of matrices, partitions and options, and the sliced-ELL
layout with ragged tiles.  Any out-of-bounds access, leak, overflow or other
undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_07769_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "native", "host_checks.cpp")] + [
    os.path.join(CSRC, f) for f in ("partition.cpp", "order.cpp", "host.cpp")]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Werror",
           *SOURCES, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all" in r.stdout and "checks passed" in r.stdout
