"""The expansion GEMM's split-K rule and slice ranges (bh_internal.h:
expand_split, split_range), host code built with hipcc and run on the CPU
(tests/host/split_check.cpp): slices partition the K-steps with lengths
differing by at most one (equal where the factor divides them), the
batch-invariant factor does not depend on the batch, the model's factor is
used only where its grid fits in two rounds of the resident workgroups, the
factors measured best at 64^3, L = 32 are the ones chosen, and a tuned factor
overrides the rule except for batch-invariant calls."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2509_01180_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_split_rule(tmp_path):
    hipcc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    exe = str(tmp_path / "split_check")
    cmd = [hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-x", "hip", "-I", CSRC,
           os.path.join(HERE, "host", "split_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=str(tmp_path))
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "ok: 0 failures" in r.stdout
