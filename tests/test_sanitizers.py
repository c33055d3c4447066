"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, CPU only) and driven through every entry point on small inputs by
tests/host/oracle_sanitize.cpp: out-of-bounds accesses, leaks and undefined
behaviour end the run with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "oracle.cpp"),
           os.path.join(ROOT, "tests", "host", "oracle_sanitize.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "0 failed expectations" in r.stdout
