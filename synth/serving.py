"""Synthetic request stream for the serving loop (inputs only).

Recipe: requests arrive as a Poisson process of rate `rate` per second; each
holds n ~ U{1..512} subtomograms of one box edge drawn uniformly from the
served boxes, matched against one of 8 resident blob templates drawn
uniformly.  Templates have U{30..80} blobs (sigma = 0.1 of the half-box, as
the other workloads); particles are a template rotated by a Haar rotation,
+/-60 degree missing wedge, noise at SNR 0.05.  To keep input synthesis off
the critical path, each (box, template) pair has a pool of pre-rendered
particles, and a request's particles are consecutive pool entries from a
random offset (its planted rotations are the pool's); starting rotations
come from a pool of Haar starts the same way.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .volumes import (add_noise, apply_wedge, blob_template, haar_quaternions,
                      matrix_to_euler_zyz, quat_to_matrix, render_blobs, seed_rng)

SERVING_CONFIG = 5
N_TEMPLATES = 8
MAX_REQUEST = 512


@dataclass
class RequestSpec:
    rid: int
    arrival: float      # seconds from the start of the run
    box: int            # box edge N
    template: int       # 0..N_TEMPLATES-1
    n: int              # particles
    offset: int         # first pool entry of its particles
    start_offset: int   # first entry of its starting rotations in the start pool


def request_stream(rate: float, duration: float, boxes, seed: int = 0,
                   max_request: int = MAX_REQUEST, pool: int = 16,
                   start_pool: int = 4096) -> list[RequestSpec]:
    """Poisson arrivals over [0, duration) with the recipe above."""
    rng = seed_rng(SERVING_CONFIG, 2, seed, 0)
    out = []
    t = 0.0
    boxes = list(boxes)
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(RequestSpec(rid=len(out), arrival=t,
                               box=int(boxes[rng.integers(len(boxes))]),
                               template=int(rng.integers(N_TEMPLATES)),
                               n=int(rng.integers(1, max_request + 1)),
                               offset=int(rng.integers(pool)),
                               start_offset=int(rng.integers(start_pool))))
    return out


def serving_templates():
    """The 8 resident templates (blob sets)."""
    out = []
    for t in range(N_TEMPLATES):
        rng = seed_rng(SERVING_CONFIG, 0, t, 0)
        n_blobs = int(rng.integers(30, 81))
        out.append(blob_template(rng, n_blobs))
    return out


def pool_rotation(box: int, template: int, j: int) -> np.ndarray:
    """Planted rotation (matrix) of pool entry j of (box, template)."""
    rng = seed_rng(SERVING_CONFIG, 1, (box * N_TEMPLATES + template) * 100003 + j, 1)
    return quat_to_matrix(haar_quaternions(rng, 1))[0]


def pool_particle(blobs, box: int, template: int, j: int, snr: float = 0.05,
                  tilt_deg: float = 60.0) -> np.ndarray:
    vol = render_blobs(blobs, box, pool_rotation(box, template, j))
    vol = apply_wedge(vol, tilt_deg)
    rng = seed_rng(SERVING_CONFIG, 1, (box * N_TEMPLATES + template) * 100003 + j, 2)
    return add_noise(vol, snr, rng).astype(np.float32)


def start_pool(n: int, restarts: int, seed: int = 0) -> np.ndarray:
    """[n, restarts, 3] Haar starting rotations as ZYZ Euler triples."""
    q = haar_quaternions(seed_rng(SERVING_CONFIG, 1, seed, 3), n * restarts)
    return matrix_to_euler_zyz(quat_to_matrix(q)).reshape(n, restarts, 3)
