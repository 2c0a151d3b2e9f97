"""Build libbh.so (HIP kernels for gfx950 + host C++) in the package directory.

    python -m paper_2509_01180_amd.build [--jobs N]

Every source under csrc/ is compiled with hipcc for gfx950 into _build/ and
linked into paper_2509_01180_amd/libbh.so.  Packed FP32 instructions are
disabled for device code.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbh.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


# Per-source flags.  The score kernels are built without machine-level loop
# invariant code motion: with it, the compiler hoists the FP64 constants of
# the sine/cosine evaluations out of every loop and, short of registers,
# spills them to scratch memory (112 bytes per lane in the ascent kernel,
# whose stores reached HBM as hundreds of MB per launch); without it the
# ascent kernel needs no scratch.
FILE_FLAGS: dict = {"bh_score.hip": ["-mllvm", "-disable-machine-licm"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def compile_one(src: str, build_dir: str = BUILD, defines=(), extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    flags = [*COMMON, *FILE_FLAGS.get(os.path.basename(src), []), *extra,
             *[f"-D{d}" for d in defines]]
    cmd = [HIPCC, *flags, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *flags, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # keep warnings visible
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build(jobs: int = 8, verbose: bool = True, out: str = LIB, build_dir: str = BUILD,
          defines=(), extra=()) -> str:
    """Compile and link the library; `defines` are extra -D build parameters
    and `extra` extra compiler flags (both for every source)."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: compile_one(s, build_dir, defines, extra), srcs))
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} from {len(srcs)} sources")
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    build(ap.parse_args().jobs)
