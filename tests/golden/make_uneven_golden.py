"""Writes uneven_config4.npz: FP64 oracle results for one sampled particle
of each box edge of the uneven-batch workload (box edges 32/48/64/96 with
bandlimits 16/24/32/40, bands every 8 up to each bandlimit, blob templates
of 30-80 blobs, wedge +/-U[50, 65] deg, SNR U[0.02, 0.2]).

    python tests/golden/make_uneven_golden.py      (about five minutes)

Only `synth` (seeded inputs) and `oracle` are called.  The 96^3, L = 40
oracle expansion alone takes about two minutes and 25 GB of host memory,
too long for a GPU test, so its results are stored here and the GPU test
(tests/test_gpu_uneven_oracle.py) regenerates the same input volumes from
their seeds and compares against them.

Per box edge N (index k in 32, 48, 64, 96), the particle is pool entry 0 of
template k.  Stored, for each N:
  tmpl_N, part_N   oracle coefficients (Sec. II-A) of the template rendered
                   at N and of the particle, complex128 [C(L_N)]
  starts_N         the P starting Euler triples of the particle [P, 3]
  best64_N         oracle march (Sec. II-C) on the FP64 coefficients:
                   (alpha, beta, gamma, score) of the best restart
  euler32_N, score32_N
                   oracle march on the FP32-rounded coefficients (the
                   values a GPU march would be handed): every restart's end
                   point [P, 3] and score [P]
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth                                   # noqa: E402
import synth.uneven as su                      # noqa: E402
from oracle import align, basis, expand        # noqa: E402

BOXES = (32, 48, 64, 96)
P, STEPS, BAND_STEP = 16, 20, 8
OUT = os.path.join(HERE, "uneven_config4.npz")


def bands_of(L: int):
    return [b for b in range(BAND_STEP, L + 1, BAND_STEP)]


def case(k: int):
    """Inputs of box index k: (N, L, template volume, particle volume, starts)."""
    N = BOXES[k]
    L = su.BOX_BANDLIMIT[N]
    blobs = su.uneven_templates()[k]
    vol, _g = su.pool_particle(blobs, N, k, 0)
    tv = synth.render_blobs(blobs, N).astype(np.float32)
    rng = synth.seed_rng(su.UNEVEN_CONFIG, 1, 7000 + k, 3)
    starts = synth.matrix_to_euler_zyz(synth.quat_to_matrix(synth.haar_quaternions(rng, P)))
    return N, L, tv, vol, starts


def fp32_round(c):
    return (c.real.astype(np.float32).astype(np.float64)
            + 1j * c.imag.astype(np.float32).astype(np.float64))


def main():
    out = {"P": np.int64(P), "steps": np.int64(STEPS), "band_step": np.int64(BAND_STEP)}
    for k, N in enumerate(BOXES):
        t0 = time.time()
        N, L, tv, vol, starts = case(k)
        idx = basis.IndexSet(L)
        c = expand.expand(np.stack([tv, vol]).astype(np.float64), idx)
        b, a = c[0], c[1]
        r64 = align.march(a, b, idx, bands_of(L), starts, STEPS)
        r32 = align.march(fp32_round(a), fp32_round(b), idx, bands_of(L), starts, STEPS)
        out[f"tmpl_{N}"] = b
        out[f"part_{N}"] = a
        out[f"starts_{N}"] = starts
        out[f"best64_{N}"] = np.append(r64["euler"][r64["best"]], r64["score"][r64["best"]])
        out[f"euler32_{N}"] = r32["euler"]
        out[f"score32_{N}"] = r32["score"]
        print(f"{N}^3 L={L}: {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
