"""Pins of the oracle's refinements of the ascent (paper Sec. II-C, Sec. III):
Hessian of Eq. (2), degree energies and the energy ratio, candidate
pruning, Newton bands.

* Hessian: central differences of the (separately pinned) gradient, and
  the SO(3) Laplacian identity Delta D^l = -l(l+1) D^l written in Euler
  coordinates, which ties the Hessian and the gradient to the degree
  scores exactly.
* Degree energies ||xi^l||_F^2: invariant under any rotation of the particle
  (D^l is unitary), equal to the Gram-matrix form sum_kk' Ga Gb, bounded by
  ||a_l||^2 ||b_l||^2.
* Energy ratio: exact values on a made-up energy profile; band selection.
* Pruning: hand-made rotations with known separations.
* Newton bands: scores never decrease; near a maximum the gradient vanishes
  to rounding within a few steps, at the point long gradient ascent finds.
"""

import numpy as np
import pytest

from oracle import align, basis, expand, score, wigner
from test_oracle_score import apply_D


@pytest.fixture(scope="module")
def coeffs():
    idx = basis.IndexSet(6)
    rng = np.random.default_rng(3)
    a = expand.real_symmetric(rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size), idx)
    b = expand.real_symmetric(rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size), idx)
    return idx, a, b


def test_hessian_matches_gradient_differences(coeffs):
    idx, a, b = coeffs
    xi = score.cross_power(a, b, idx, 6)
    e = np.array([[0.3, 1.1, -0.7], [2.0, 0.4, 1.0], [-2.5, 2.8, 0.1]])
    _S, _G, H = score.score_grad_hess(xi, e)
    h = 1e-5
    scale = score.cs_bound(a, b, idx, 6) * 6 * 7
    for k in range(3):
        ep, em = e.copy(), e.copy()
        ep[:, k] += h
        em[:, k] -= h
        fd = (score.score_grad(xi, ep)[1] - score.score_grad(xi, em)[1]) / (2 * h)
        assert np.max(np.abs(fd - H[:, :, k])) <= 1e-8 * scale
    assert np.allclose(H, np.transpose(H, (0, 2, 1)))


@pytest.mark.parametrize("beta", [0.2, 1.3, 2.9])
def test_laplacian_identity(coeffs, beta):
    """Delta S = H_bb + cot(b) g_b + (H_aa + H_gg - 2 cos(b) H_ag) / sin^2(b)
    equals -sum_l l(l+1) S_l (Delta D^l = -l(l+1) D^l on SO(3))."""
    idx, a, b = coeffs
    xi = score.cross_power(a, b, idx, 6)
    e = np.array([[0.7, beta, -1.9]])
    S, G, H = score.score_grad_hess(xi, e)
    cb, sb = np.cos(beta), np.sin(beta)
    lap = H[0, 1, 1] + cb / sb * G[0, 1] + (H[0, 0, 0] + H[0, 2, 2] - 2 * cb * H[0, 0, 2]) / sb ** 2
    ref = 0.0
    for l in range(len(xi)):
        only = [x if j == l else np.zeros_like(x) for j, x in enumerate(xi)]
        ref += -l * (l + 1) * score.score(only, e)[0]
    assert abs(lap - ref) <= 1e-10 * score.cs_bound(a, b, idx, 6) * 42


def test_degree_energy_invariants(coeffs):
    idx, a, b = coeffs
    L = 6
    E = score.degree_energy(a, b, idx, L)
    # rotation of the particle leaves every ||xi^l||_F unchanged
    Er = score.degree_energy(apply_D(a, idx, (0.4, 2.2, -1.1)), b, idx, L)
    np.testing.assert_allclose(Er, E, rtol=1e-12, atol=1e-14 * E.max())
    # Gram form: ||A^H B||_F^2 = sum_{k,k'} (A^H A)... written per degree
    keep = score.band_mask(idx, L)
    for l in range(L + 1):
        rows = [off for (ll, _k, _lam, _c), off in zip(idx.radial, idx.offset) if ll == l and keep[off]]
        A = np.array([a[o:o + 2 * l + 1] for o in rows])       # [K, 2l+1]
        Bm = np.array([b[o:o + 2 * l + 1] for o in rows])
        Ga = A @ A.conj().T                                     # Ga[k,k'] = sum_m a_km conj(a_k'm)
        Gb = Bm @ Bm.conj().T
        assert abs(np.sum(Ga * Gb.conj()) - E[l]) <= 1e-12 * max(E[l], 1e-300) + 1e-14
        assert E[l] <= np.sum(np.abs(A) ** 2) * np.sum(np.abs(Bm) ** 2) * (1 + 1e-12)


def test_energy_ratio_and_band_selection():
    E = np.array([4.0, 2.0, 1.0, 0.5, 0.25, 0.25])      # total 8
    r = score.energy_ratio(E)
    np.testing.assert_allclose(r, [0.5, 0.25, 0.125, 0.0625, 0.03125, 0.0])
    assert score.select_bands(r, [0.3, 0.1, 0.05]) == [1, 3, 4]
    assert score.select_bands(r, [0.0]) == [5]
    assert score.select_bands(r, [0.5, 0.5]) == [0]
    assert np.all(score.energy_ratio(np.zeros(4)) == 0)


def test_batch_band_selection():
    """The batch's band per threshold: at least half the particles' ratio
    curves at or below tau.  Pinned by hand on made-up curves, by the
    median formulation (for an odd batch the band of the median ratio
    curve, taken pointwise in L) and by the lower median of the
    per-particle choices."""
    r = np.array([[0.5, 0.2, 0.05, 0.0],
                  [0.6, 0.4, 0.1, 0.0],
                  [0.3, 0.1, 0.01, 0.0]])
    # tau 0.1: per-particle choices 2, 2, 1 -> at L=1 one curve of three is <= 0.1, at L=2 all
    assert score.select_bands_batch(r, [0.1]) == [2]
    # tau 0.2: choices 1, 2, 1 -> L=1; tau 0: every curve reaches 0 at L=3; tau 1: L=0
    assert score.select_bands_batch(r, [0.2, 0.0, 1.0]) == [1, 3, 0]
    rng = np.random.default_rng(3)
    for B in (1, 5, 7, 8, 20):
        E = rng.exponential(size=(B, 13)) * np.exp(-0.4 * np.arange(13))
        R = np.stack([score.energy_ratio(e) for e in E])
        taus = [0.3, 0.05, 0.01, 0.001]
        got = score.select_bands_batch(R, taus)
        per = np.array([[score.select_bands(R[b], [t])[0] for t in taus] for b in range(B)])
        lower_median = np.sort(per, axis=0)[(B - 1) // 2]
        assert got == list(lower_median)
        if B % 2:
            med = np.median(R, axis=0)
            assert got == [score.select_bands(med, [t])[0] for t in taus]


def test_prune_candidates_rules():
    # rotations about z by these angles (degrees): separations are exact
    ang = np.radians([0.0, 3.0, 40.0, 41.0, 90.0, 200.0])
    x = np.stack([[t, 0.0, 0.0] for t in ang])
    S = np.array([5.0, 4.0, 3.0, 6.0, 1.0, 3.0])
    sep = np.radians(10.0)
    # order by score: 3 (41), 0 (0), 1 (3), 2 (40), 5 (200), 4 (90)  [2 before 5: tie, lower index]
    # 1 is within 10 deg of 0, 2 within 10 deg of 3
    assert list(align.prune_candidates(x, S, 3, sep)) == [3, 0, 5]
    assert list(align.prune_candidates(x, S, 4, sep)) == [3, 0, 5, 4]
    # only four distinct maxima: the fifth and sixth slots take the skipped ones in order
    assert list(align.prune_candidates(x, S, 6, sep)) == [3, 0, 5, 4, 1, 2]
    # zero separation keeps the score order
    assert list(align.prune_candidates(x, S, 6, 0.0)) == [3, 0, 1, 2, 5, 4]


def _problem():
    idx = basis.IndexSet(8)
    rng = np.random.default_rng(11)
    b = expand.real_symmetric(rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size), idx)
    g = np.array([0.9, 1.2, -0.4])
    a = apply_D(b, idx, g)          # particle = template rotated by g: maximum at g^{-1}
    return idx, a, b, wigner.matrix_to_euler(wigner.euler_to_matrix(*g).T)


def test_newton_band_converges_and_is_monotone():
    idx, a, b, top = _problem()
    rng = np.random.default_rng(5)
    starts = top[None] + 0.05 * rng.standard_normal((4, 3))
    r = align.march(a, b, idx, (8,), starts, 8, newton_bands=1, trace=True)
    for h in r["trace"]:
        assert np.all(np.diff(h, axis=0) >= 0)
    xi = score.cross_power(a, b, idx, 8)
    _S, G = score.score_grad(xi, r["euler"])
    assert np.max(np.abs(G)) <= 1e-9 * score.cs_bound(a, b, idx, 8)
    # the planted maximum, which a long gradient ascent also reaches
    rg = align.march(a, b, idx, (8,), starts, 200)
    for e1, e2 in zip(r["euler"], rg["euler"]):
        assert wigner.geodesic_deg(wigner.euler_to_matrix(*e1), wigner.euler_to_matrix(*e2)) < 1e-3
        assert wigner.geodesic_deg(wigner.euler_to_matrix(*e1), wigner.euler_to_matrix(*top)) < 1e-6


def test_keep_prunes_after_first_band():
    idx, a, b, _top = _problem()
    rng = np.random.default_rng(8)
    starts = np.stack([wigner.matrix_to_euler(m) for m in
                       [wigner.euler_to_matrix(*(rng.uniform(-3, 3, 3))) for _ in range(12)]])
    full = align.march(a, b, idx, (4,), starts, 10)
    sel = align.prune_candidates(full["euler"], full["score"], 3, np.radians(5.0))
    r = align.march(a, b, idx, (4, 8), starts, 10, keep=3, min_sep=np.radians(5.0))
    assert r["euler"].shape == (3, 3)
    cont = align.march(a, b, idx, (8,), full["euler"][sel], 10)
    np.testing.assert_array_equal(r["euler"], cont["euler"])
    np.testing.assert_array_equal(r["score"], cont["score"])
