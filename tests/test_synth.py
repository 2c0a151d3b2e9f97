"""Checks of the seeded synthetic-input generator (no method arithmetic)."""

import numpy as np

import synth


def test_rotations_valid_and_euler_roundtrip():
    rng = synth.seed_rng(9, 1, 0, 3)
    R = synth.quat_to_matrix(synth.haar_quaternions(rng, 100))
    np.testing.assert_allclose(R @ np.transpose(R, (0, 2, 1)), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    e = synth.matrix_to_euler_zyz(R)
    np.testing.assert_allclose(synth.euler_zyz_to_matrix(e), R, atol=1e-12)
    # Haar: E[R] = 0
    assert np.abs(R.mean(axis=0)).max() < 0.25


def test_render_blobs_direct():
    rng = synth.seed_rng(9, 0, 0, 0)
    bl = synth.blob_template(rng, 7)
    assert np.all(np.linalg.norm(bl.centres, axis=1) <= 0.8)
    g = synth.quat_to_matrix(synth.haar_quaternions(rng, 1))[0]
    N = 10
    vol = synth.render_blobs(bl, N, g)
    x = (np.arange(N) - (N - 1) / 2) * 2 / N
    for (i, j, k) in [(0, 0, 0), (3, 5, 7), (9, 2, 4)]:
        p = np.array([x[i], x[j], x[k]])
        ref = sum(A * np.exp(-np.sum((p - g @ c) ** 2) / (2 * bl.sigma ** 2))
                  for A, c in zip(bl.amps, bl.centres))
        assert abs(vol[i, j, k] - ref) < 1e-13


def test_wedge_and_noise():
    N = 32
    m = synth.wedge_mask(N, 60.0)
    kx = np.fft.fftfreq(N)[:, None, None]
    kz = np.fft.rfftfreq(N)[None, None, :]
    missing = np.broadcast_to(np.abs(kz) > np.tan(np.radians(60)) * np.abs(kx) + 1e-9, m.shape)
    assert np.all(m[missing] == 0) and np.all(m[~missing] == 1)
    assert 0.5 < m.mean() < 0.8
    rng = np.random.default_rng(0)
    v = rng.standard_normal((N, N, N))
    w = synth.apply_wedge(v)
    np.testing.assert_allclose(synth.apply_wedge(w), w, atol=1e-12)        # projection
    n = synth.add_noise(np.zeros((N, N, N)) + w, 0.1, np.random.default_rng(1)) - w
    assert abs(np.var(n) / np.var(w) - 10.0) < 0.3


def test_workload_deterministic():
    w = synth.CONFIG1
    a = w.particle(3)
    b = w.particle(3)
    assert a.dtype == np.float32 and a.shape == (32, 32, 32)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, w.particle(4))
    s = w.starts(0)
    assert s.shape == (w.restarts, 3)
    np.testing.assert_array_equal(s, w.starts(0))
