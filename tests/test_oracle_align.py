"""Pins of the oracle's frequency-marching ascent (paper Sec. II-C).

* Ascent direction: the natural gradient in Euler coordinates must map to
  the body-frame gradient of SO(3) (checked with rotation matrices only).
* Planted rotation: a noise-free, wedge-free particle t(g*^{-1} x) is
  aligned back by g*^{-1}.
* The accept/reject rule makes the score non-decreasing within a band.
* Degenerate inputs (zero particle) do not produce NaN.
"""

import numpy as np
import pytest

import synth
from oracle import align, basis, expand, score, wigner


def skew(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def expm_so3(w):
    th = np.linalg.norm(w)
    if th == 0:
        return np.eye(3)
    K = skew(w / th)
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


@pytest.mark.parametrize("beta", [0.05, 0.7, 1.6, 2.9])
def test_natural_gradient_is_body_gradient(beta):
    rng = np.random.default_rng(int(beta * 100))
    A = rng.standard_normal((3, 3))
    S = lambda R: np.trace(A @ R)                       # smooth function on SO(3)
    e = np.array([0.4, beta, -1.3])
    h = 1e-6
    grad_e = np.zeros(3)
    for j in range(3):
        d = np.zeros(3)
        d[j] = h
        grad_e[j] = (S(wigner.euler_to_matrix(*(e + d))) - S(wigner.euler_to_matrix(*(e - d)))) / (2 * h)
    R = wigner.euler_to_matrix(*e)
    grad_body = np.array([(S(R @ expm_so3(h * np.eye(3)[i])) - S(R @ expm_so3(-h * np.eye(3)[i]))) / (2 * h)
                          for i in range(3)])
    de = align.ascent_direction(e[None], grad_e[None])[0]
    # body angular velocity produced by moving along de
    Om = R.T @ (wigner.euler_to_matrix(*(e + h * de)) - wigner.euler_to_matrix(*(e - h * de))) / (2 * h)
    omega = np.array([Om[2, 1], Om[0, 2], Om[1, 0]])
    np.testing.assert_allclose(omega, grad_body, rtol=1e-5, atol=1e-6 * np.abs(grad_body).max())


@pytest.fixture(scope="module")
def cfg1():
    w = synth.CONFIG1
    idx = basis.IndexSet(w.L_max)
    b = expand.expand(w.template_volume().astype(np.float64), idx)
    return w, idx, b


@pytest.mark.parametrize("i", [0, 2])
def test_planted_rotation_recovered(cfg1, i):
    w, idx, b = cfg1
    a = expand.expand(w.particle(i, wedge=False, noise=False).astype(np.float64), idx)
    r = align.march(a, b, idx, w.bands, w.starts(i), w.steps, trace=True)
    e = r["euler"][r["best"]]
    err = wigner.geodesic_deg(wigner.euler_to_matrix(*e), w.truth(i).T)
    assert err < 0.05
    for band in r["trace"]:
        assert np.all(np.diff(band, axis=0) >= 0)       # accept/reject monotonicity


def test_noisy_particle_reaches_global_max(cfg1):
    # With wedge and noise the answer is the maximiser of the noisy score,
    # which ascent from the truth also reaches.
    w, idx, b = cfg1
    a = expand.expand(w.particle(1).astype(np.float64), idx)
    r = align.march(a, b, idx, w.bands, w.starts(1), w.steps)
    et = wigner.matrix_to_euler(w.truth(1).T)
    r2 = align.march(a, b, idx, (w.bands[-1],), et[None], 40)
    assert r["score"][r["best"]] >= r2["score"][0] - 1e-9 * abs(r2["score"][0])
    e1 = wigner.euler_to_matrix(*r["euler"][r["best"]])
    e2 = wigner.euler_to_matrix(*r2["euler"][0])
    assert wigner.geodesic_deg(e1, e2) < 0.05


def test_zero_particle_and_ties(cfg1):
    w, idx, b = cfg1
    a = np.zeros_like(b)
    starts = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [1.0, 2.0, 3.0]])
    r = align.march(a, b, idx, w.bands, starts, 5)
    assert np.all(np.isfinite(r["euler"])) and np.all(r["score"] == 0)
    assert r["best"] == 0
    np.testing.assert_allclose(r["euler"], align.wrap_many(starts))
