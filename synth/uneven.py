"""Synthetic uneven batch (inputs only): subtomograms of several box sizes.

Recipe: box edges {32, 48, 64, 96} in equal shares, each with its own
bandlimit (16, 24, 32, 40); 4 blob templates with U{30..80} blobs; each
particle a template rotated by a Haar rotation, with a missing wedge of
+/- U[50, 65] degrees and noise at SNR U[0.02, 0.2] drawn per particle.  A
pool of pre-rendered particles per (box, template) is tiled to the batch
size, keeping input synthesis short; every particle gets its own starts.
"""

from __future__ import annotations

import numpy as np

from .volumes import (add_noise, apply_wedge, blob_template, haar_quaternions, quat_to_matrix,
                      render_blobs, seed_rng)

UNEVEN_CONFIG = 4
BOX_BANDLIMIT = {32: 16, 48: 24, 64: 32, 96: 40}
N_TEMPLATES = 4


def uneven_templates():
    out = []
    for t in range(N_TEMPLATES):
        rng = seed_rng(UNEVEN_CONFIG, 0, t, 0)
        out.append(blob_template(rng, int(rng.integers(30, 81))))
    return out


def pool_particle(blobs, box: int, template: int, j: int):
    """Pool entry j of (box, template): (volume float32, planted rotation)."""
    key = (box * N_TEMPLATES + template) * 100003 + j
    g = quat_to_matrix(haar_quaternions(seed_rng(UNEVEN_CONFIG, 1, key, 1), 1))[0]
    rng = seed_rng(UNEVEN_CONFIG, 1, key, 2)
    tilt = rng.uniform(50.0, 65.0)
    snr = rng.uniform(0.02, 0.2)
    vol = apply_wedge(render_blobs(blobs, box, g), tilt)
    return add_noise(vol, snr, rng).astype(np.float32), g
