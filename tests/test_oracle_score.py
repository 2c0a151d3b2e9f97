"""Pins of the oracle's expansion, cross-power and score (paper Sec. II-A/B).

* Expansion + Wigner D: for the 24 rotations of the cube, rotating a
  cell-centred voxel volume is an exact permutation, so the voxel
  quadrature must satisfy a(R_g f) = D(g) a(f) to rounding.
* Score: Eq. (1) at zero shift, integrated by an exact product quadrature
  with the rotated function evaluated at rotated points, must equal the
  oracle's Eq. (2) for arbitrary rotations.
* Gradient: central differences.  Self-correlation: maximal at the
  identity with value ||a||^2; |C| bounded by Cauchy-Schwarz.
"""

import itertools

import numpy as np
import pytest

from oracle import basis, expand, score, wigner
from test_oracle_basis import exact_ball_quadrature


def cube_rotations():
    out = []
    for p in itertools.permutations(range(3)):
        for s in itertools.product([1, -1], repeat=3):
            M = np.zeros((3, 3))
            for i in range(3):
                M[i, p[i]] = s[i]
            if np.linalg.det(M) > 0:
                out.append(M)
    return out


def rotate_voxels(f, g):
    """(R_g f)(x) = f(g^{-1} x) for a cube rotation g on the cell-centred grid."""
    N = f.shape[0]
    c = np.arange(N) - (N - 1) / 2.0
    pos = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1)
    src = np.rint(pos @ g + (N - 1) / 2.0).astype(int)     # row-vector form of g^T x
    return f[src[..., 0], src[..., 1], src[..., 2]]


def apply_D(a, idx, e):
    out = np.zeros_like(a)
    for (l, _k, _lam, _c), off in zip(idx.radial, idx.offset):
        out[off:off + 2 * l + 1] = wigner.wigner_D(l, *e) @ a[off:off + 2 * l + 1]
    return out


@pytest.fixture(scope="module")
def small():
    idx = basis.IndexSet(5)
    rng = np.random.default_rng(21)
    f = rng.standard_normal((12, 12, 12))
    t = rng.standard_normal((12, 12, 12))
    return idx, f, t, expand.expand(f, idx), expand.expand(t, idx)


def test_cube_rotations_exact(small):
    idx, f, _t, a, _b = small
    rots = cube_rotations()
    assert len(rots) == 24
    for g in rots:
        e = wigner.matrix_to_euler(g)
        ap = expand.expand(rotate_voxels(f, g), idx)
        np.testing.assert_allclose(ap, apply_D(a, idx, e), atol=1e-13 * np.abs(a).max())


def test_real_symmetry(small):
    idx, _f, _t, a, _b = small
    for (l, _k, _lam, _c), off in zip(idx.radial, idx.offset):
        blk = a[off:off + 2 * l + 1]
        ms = np.arange(-l, l + 1)
        np.testing.assert_allclose(blk[::-1], (-1.0) ** ms * np.conj(blk), atol=1e-14)


def test_score_cube_rotations_voxel_inner_product(small):
    # C(g) over the band = sum_c conj(b_c) a_c(R_g f)  (Parseval, exact for cube g).
    idx, f, _t, a, b = small
    for L in (2, 5):
        keep = score.band_mask(idx, L)
        xi = score.cross_power(a, b, idx, L)
        for g in cube_rotations()[::3]:
            e = wigner.matrix_to_euler(g)
            ap = expand.expand(rotate_voxels(f, g), idx)
            ref = np.real(np.vdot(b[keep], ap[keep]))
            assert abs(score.score(xi, e[None])[0] - ref) < 1e-12 * np.abs(a).max() * np.abs(b).max() * idx.size


def _random_real_coeffs(idx, rng):
    c = rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)
    return expand.real_symmetric(c, idx)


def test_score_equals_eq1_by_quadrature():
    """Eq. (1) (zero shift) for band-limited t, f == Eq. (2) with xi = conj(b) a^T."""
    idx = basis.IndexSet(4)
    rng = np.random.default_rng(7)
    a = _random_real_coeffs(idx, rng)
    b = _random_real_coeffs(idx, rng)
    X, W = exact_ball_quadrature(nr=60, nt=16, nphi=24)
    t = np.real(basis.psi(idx, X) @ b)
    xi = score.cross_power(a, b, idx, 4)
    for _ in range(4):
        e = np.array([rng.uniform(-np.pi, np.pi), rng.uniform(0, np.pi), rng.uniform(-np.pi, np.pi)])
        g = wigner.euler_to_matrix(*e)
        f_rot = np.real(basis.psi(idx, X @ g) @ a)        # f(g^{-1} x)
        C = np.sum(W * t * f_rot)
        assert abs(C - score.score(xi, e[None])[0]) < 1e-12 * np.linalg.norm(a) * np.linalg.norm(b)


def test_score_imaginary_part_vanishes(small):
    idx, _f, _t, a, b = small
    xi = score.cross_power(a, b, idx, 5)
    e = np.array([0.4, 1.1, -2.0])
    tot = sum(np.sum(x * wigner.wigner_D(l, *e)) for l, x in enumerate(xi))
    assert abs(tot.imag) < 1e-12 * abs(tot.real)


def test_gradient_finite_difference(small):
    idx, _f, _t, a, b = small
    xi = score.cross_power(a, b, idx, 5)
    rng = np.random.default_rng(4)
    E = np.column_stack([rng.uniform(-np.pi, np.pi, 6), rng.uniform(0.05, np.pi - 0.05, 6),
                         rng.uniform(-np.pi, np.pi, 6)])
    S, G = score.score_grad(xi, E)
    h = 1e-6
    for j in range(3):
        dE = np.zeros(3)
        dE[j] = h
        fd = (score.score(xi, E + dE) - score.score(xi, E - dE)) / (2 * h)
        np.testing.assert_allclose(G[:, j], fd, rtol=1e-7, atol=1e-8 * np.abs(S).max())


def test_self_correlation_max_and_cs_bound(small):
    idx, f, _t, a, _b = small
    L = 5
    xi = score.cross_power(a, a, idx, L)
    keep = score.band_mask(idx, L)
    s0 = score.score(xi, np.zeros((1, 3)))[0]
    assert abs(s0 - np.sum(np.abs(a[keep]) ** 2)) < 1e-12 * s0
    rng = np.random.default_rng(8)
    E = np.column_stack([rng.uniform(-np.pi, np.pi, 40), rng.uniform(0, np.pi, 40),
                         rng.uniform(-np.pi, np.pi, 40)])
    s = score.score(xi, E)
    assert np.all(s <= s0 + 1e-12)
    assert np.all(np.abs(s) <= score.cs_bound(a, a, idx, L) * (1 + 1e-12))


def test_cross_power_band_prefix(small):
    idx, _f, _t, a, b = small
    for L in range(0, 6):
        xi = score.cross_power(a, b, idx, L)
        assert len(xi) == L + 1
        keep = score.band_mask(idx, L)
        tot = sum(np.trace(x) for x in xi)
        # trace of xi summed over l = <b, a> restricted to the band
        assert abs(tot - np.vdot(b[keep], a[keep])) < 1e-13 * np.linalg.norm(a) * np.linalg.norm(b)
