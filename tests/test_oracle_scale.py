"""Pins of the oracle's absolute scales (paper Sec. II-A, Sec. II-C).

The other expansion pins are linear or scale-invariant (rotation
covariance, symmetry, self-correlation), so they would not notice a wrong
constant factor.  These tests fix the scale of two functions against values
that do not come from the oracle:

* ``expand.expand``: the coefficients of the L2(B)-orthonormal basis,
  a_klm = <f, psi_klm>, approximated by the voxel midpoint rule with cell
  volume h^3.  For f = 1, f = z and f = x + i y the inner products have
  closed forms (below); the voxel rule must reproduce them.  On the voxel
  grid the sampled basis functions themselves must expand to (nearly) the
  identity, and a band-limited f = sum_c c_c psi_c back to its c.
* ``score.curvature_weight``: W_L = sum_l l(l+1) ||a_l|| ||b_l|| bounds the
  magnitude of the SO(3) Laplacian of the band-L score, Delta S(g) =
  -sum_l l(l+1) S_l(g) (Delta D^l = -l(l+1) D^l).  At the planted maximum of
  a particle that is an exact rotation of the template every degree score
  equals ||b_l||^2, so the bound is attained: W_L = -Delta S.  The Laplacian
  is taken from the oracle's Hessian and gradient, which are pinned by
  central differences elsewhere.
"""

import numpy as np
import pytest
from scipy import special

from oracle import basis, expand, score, wigner
from test_oracle_score import apply_D


def _blocks(idx, l):
    return [(k, lam, off) for (ll, k, lam, _c), off in zip(idx.radial, idx.offset) if ll == l]


@pytest.mark.parametrize("N", [32, 48])
def test_expand_constant_closed_form(N):
    """f = 1: a_k00 = c_k0 Y_0^0 4 pi int_0^1 j_0(k pi r) r^2 dr.

    With lambda_0k = k pi, |j_1(k pi)| = 1/(k pi), so c_k0 = sqrt(2) k pi, and
    int_0^1 sin(k pi r) r dr / (k pi) = (-1)^(k+1) / (k pi)^2; hence
    a_k00 = (-1)^(k+1) sqrt(8 pi) / (k pi), and every a_k0m with m != 0 is 0
    for l = 0 trivially.
    """
    idx = basis.IndexSet(4)
    a = expand.expand(np.ones((N, N, N)), idx)
    for k, lam, off in _blocks(idx, 0):
        ref = (-1.0) ** (k + 1) * np.sqrt(8 * np.pi) / (k * np.pi)
        assert abs(lam - k * np.pi) < 1e-12
        assert abs(a[off] - ref) <= 1e-4 * abs(ref), (k, a[off], ref)


@pytest.mark.parametrize("N", [32, 48])
def test_expand_linear_closed_form(N):
    """f = z and f = x + i y (degree 1, Condon-Shortley phase).

    int_0^1 r^3 j_1(lam r) dr = j_2(lam)/lam (from d/dx[x^3 j_2(x)] = x^3 j_1(x)),
    and c_k1 = sqrt(2)/|j_2(lam)|.  With int cos(t) Y_1^0 dOmega = sqrt(4 pi/3)
    and int sin(t) e^{i p} conj(Y_1^1) dOmega = -sqrt(8 pi/3):
      f = z:       a_k10 = s sqrt(8 pi/3) / lam,       a_k1,+-1 = 0
      f = x + i y: a_k11 = -s sqrt(16 pi/3) / lam,     a_k1,-1 = a_k10 = 0
    with s = sign(j_2(lam_1k)).
    """
    idx = basis.IndexSet(4)
    h, xyz, _ball = basis.grid(N)
    fz = xyz[..., 2]
    fxy = xyz[..., 0] + 1j * xyz[..., 1]
    a = expand.expand(np.stack([fz, fxy]), idx)
    for _k, lam, off in _blocks(idx, 1):
        s = np.sign(special.spherical_jn(2, lam))
        rz = s * np.sqrt(8 * np.pi / 3) / lam
        rxy = -s * np.sqrt(16 * np.pi / 3) / lam
        got_z, got_xy = a[0, off:off + 3], a[1, off:off + 3]       # m = -1, 0, 1
        np.testing.assert_allclose(got_z, [0, rz, 0], atol=1e-4 * abs(rz))
        np.testing.assert_allclose(got_xy, [0, 0, rxy], atol=1e-4 * abs(rxy))


@pytest.fixture(scope="module")
def sampled_basis():
    N, L = 32, 8
    idx = basis.IndexSet(L)
    _h, xyz, _ball = basis.grid(N)
    P = basis.psi(idx, xyz)                 # [N, N, N, C], zero outside the ball
    return idx, P


def test_voxel_gram_near_identity(sampled_basis):
    """Expanding the sampled psi_c gives the voxel Gram matrix h^3 Psi^H Psi.
    It is I up to the voxel rule's error (6.1e-4 in 2-norm at 32^3, L = 8)."""
    idx, P = sampled_basis
    G = expand.expand(np.moveaxis(P, -1, 0), idx)           # G[c', c] = <psi_c', psi_c>_h
    dev = np.linalg.norm(G - np.eye(idx.size), 2)
    assert dev < 2e-3, dev
    # The diagonal alone is 1 to the same accuracy (a wrong h power moves it by N/2).
    assert np.max(np.abs(np.diag(G).real - 1)) < 2e-3


def test_band_limited_round_trip(sampled_basis):
    """f = sum_c c_c psi_c (real f) expands back to c, and Parseval holds:
    h^3 sum_v f(x_v)^2 = ||c||^2 up to the voxel rule's error."""
    idx, P = sampled_basis
    rng = np.random.default_rng(7)
    c = expand.real_symmetric(rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size), idx)
    f = P @ c
    assert np.max(np.abs(f.imag)) < 1e-12 * np.max(np.abs(f.real))
    f = f.real
    a = expand.expand(f, idx)
    assert np.linalg.norm(a - c) <= 2e-3 * np.linalg.norm(c)
    h = 2.0 / f.shape[0]
    assert abs(h ** 3 * np.sum(f * f) - np.linalg.norm(c) ** 2) <= 4e-3 * np.linalg.norm(c) ** 2


def _laplacian(xi, e):
    """Delta S in ZYZ Euler coordinates from the oracle's gradient and Hessian."""
    _S, G, H = score.score_grad_hess(xi, e[None])
    cb, sb = np.cos(e[1]), np.sin(e[1])
    return H[0, 1, 1] + cb / sb * G[0, 1] + (H[0, 0, 0] + H[0, 2, 2] - 2 * cb * H[0, 0, 2]) / sb ** 2


@pytest.mark.parametrize("L", [3, 6])
def test_curvature_weight_attained_at_planted_maximum(L):
    idx = basis.IndexSet(6)
    rng = np.random.default_rng(31)
    b = expand.real_symmetric(rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size), idx)
    g0 = np.array([0.8, 1.3, -2.1])
    a = apply_D(b, idx, g0)                          # particle = template rotated by g0
    top = wigner.matrix_to_euler(wigner.euler_to_matrix(*g0).T)     # maximum at g0^{-1}
    xi = score.cross_power(a, b, idx, L)
    W = score.curvature_weight(a, b, idx, L)
    # the degree scores at the maximum are ||b_l||^2 over the band
    na, nb = score.band_norms(a, b, idx, L)
    np.testing.assert_allclose(na, nb, rtol=1e-12)
    for l in range(L + 1):
        only = [x if j == l else np.zeros_like(x) for j, x in enumerate(xi)]
        assert abs(score.score(only, top[None])[0] - nb[l] ** 2) <= 1e-11 * max(nb[l] ** 2, 1e-300)
    lap = _laplacian(xi, top)
    assert lap < 0
    assert abs(W + lap) <= 1e-9 * W, (W, -lap)
    # brute force: W is the sum over the band's degrees of l(l+1) ||a_l|| ||b_l||
    keep = score.band_mask(idx, L)
    brute = 0.0
    for l in range(L + 1):
        sel = keep & (idx.l == l)
        brute += l * (l + 1) * np.linalg.norm(a[sel]) * np.linalg.norm(b[sel])
    assert abs(W - brute) <= 1e-12 * brute


def test_curvature_weight_bounds_laplacian():
    """|Delta S(g)| <= W_L at arbitrary rotations, for unrelated a and b."""
    idx = basis.IndexSet(6)
    rng = np.random.default_rng(5)
    a = expand.real_symmetric(rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size), idx)
    b = expand.real_symmetric(rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size), idx)
    L = 6
    xi = score.cross_power(a, b, idx, L)
    W = score.curvature_weight(a, b, idx, L)
    for _ in range(20):
        e = np.array([rng.uniform(-np.pi, np.pi), rng.uniform(0.2, np.pi - 0.2), rng.uniform(-np.pi, np.pi)])
        assert abs(_laplacian(xi, e)) <= W * (1 + 1e-12)
