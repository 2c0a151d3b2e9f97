"""Pins of the oracle's shift search (Sec. II-C: a grid of shifts, the
rotation maximised for each).

* The voxel shift equals sampling the shifted function: a blob volume
  rendered with its centres moved by -d h, shifted by d, is the unshifted
  rendering wherever the shift does not cross the box edge.
* A particle planted with a known voxel shift and rotation is recovered:
  the best shift is the planted one and the rotation is within a degree.
"""

import numpy as np

import synth
from oracle import align, basis, expand, wigner


def _shifted_blobs(bl, dvox, N, rot=None):
    c = bl.centres if rot is None else bl.centres @ np.asarray(rot).T
    return synth.volumes.Blobs(centres=c + np.asarray(dvox) * (2.0 / N), amps=bl.amps,
                               sigma=bl.sigma)


def test_shift_is_translation_of_samples():
    N = 16
    rng = np.random.default_rng(2)
    bl = synth.blob_template(rng, 6, radius=0.4)
    d = (1, -2, 0)
    moved = synth.render_blobs(_shifted_blobs(bl, -np.array(d), N), N)   # t(x + d h)
    ref = synth.render_blobs(bl, N)
    got = expand.shift_volume(moved, (-d[0], -d[1], -d[2]))              # back by -d
    inner = (slice(2, N - 2),) * 3
    np.testing.assert_allclose(got[inner], ref[inner], atol=1e-12)
    # the shift of zero is the identity; shifting out of the box leaves zeros
    np.testing.assert_array_equal(expand.shift_volume(ref, (0, 0, 0)), ref)
    assert not np.any(expand.shift_volume(ref, (N, 0, 0)))


def test_planted_shift_and_rotation_recovered():
    N, L = 20, 6
    idx = basis.IndexSet(L)
    rng = np.random.default_rng(9)
    bl = synth.blob_template(rng, 8, radius=0.55)
    g = synth.quat_to_matrix(synth.haar_quaternions(rng, 1))[0]
    s_true = (1, 0, -1)
    # f(x) = t(g^{-1}(x - s h)): shifting f by s undoes the translation
    f = synth.render_blobs(_shifted_blobs(bl, s_true, N, rot=g), N)
    b = expand.expand(synth.render_blobs(bl, N), idx)
    shifts = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 0, -1), (-1, 0, 1)]
    starts = synth.matrix_to_euler_zyz(synth.quat_to_matrix(synth.haar_quaternions(rng, 16)))
    e, s, si = align.align_shifts(f, b, idx, shifts, (3, 6), starts, 12)
    assert tuple(shifts[si]) == s_true
    assert wigner.geodesic_deg(wigner.euler_to_matrix(*e), g.T) < 1.5
