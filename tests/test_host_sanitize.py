"""The host table builders (bh_tables.cpp: Bessel zeros, index sets, band
tables, work splits, voxel lists, the union of launch intervals) under AddressSanitizer and
UndefinedBehaviorSanitizer with bounds-checked standard containers, built
with g++ for the host only (no GPU code), and their invariants checked
(tests/host/tables_check.cpp)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2509_01180_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tables_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D_GLIBCXX_ASSERTIONS",
           "-I", CSRC, os.path.join(HERE, "host", "tables_check.cpp"),
           os.path.join(CSRC, "bh_tables.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "ok: 0 failures" in r.stdout
