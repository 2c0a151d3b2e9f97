"""Pins of the oracle's ball-harmonic basis (paper Sec. II-A) to mathematics.

Bessel zeros against closed forms and mpmath; normalisation against
Gauss-Legendre quadrature of the radial integral; spherical harmonics
against textbook closed forms and the addition theorem; orthonormality of
psi_klm against an exact product quadrature; voxel counts by integer brute
force.
"""

import math

import mpmath
import numpy as np
import pytest
from scipy import special

from oracle import basis


def test_zeros_l0_closed_form():
    # j_0(x) = sin(x)/x: zeros at k*pi.
    z = basis.bessel_zeros(0, 40.0)
    k = np.arange(1, len(z) + 1)
    assert len(z) == 12
    np.testing.assert_allclose(z, k * np.pi, rtol=0, atol=1e-13)


def test_zeros_l1_tan_equation():
    # j_1(x) = sin x / x^2 - cos x / x = 0  <=>  tan x = x.
    z = basis.bessel_zeros(1, 30.0)
    assert len(z) == 9
    np.testing.assert_allclose(np.tan(z), z, rtol=1e-11)
    for k, zk in enumerate(z):
        # root of x cos x - sin x in ((k+1) pi, (k+3/2) pi), bracketed
        ref = mpmath.findroot(lambda t: t * mpmath.cos(t) - mpmath.sin(t),
                              ((k + 1) * mpmath.pi + 0.1, (k + 1.5) * mpmath.pi),
                              solver="illinois")
        assert abs(zk - float(ref)) < 1e-13 * zk


@pytest.mark.parametrize("l", [0, 1, 2, 5, 11, 20, 33, 42])
def test_zeros_against_mpmath(l):
    # lambda_lk = j_{l+1/2, k} (zeros of the cylinder function J_{l+1/2}).
    z = basis.bessel_zeros(l, l + 25.0)
    assert len(z) >= 4
    for k in range(1, 5):
        ref = float(mpmath.besseljzero(l + 0.5, k))
        assert abs(z[k - 1] - ref) < 1e-12 * ref


def test_zeros_interlace():
    for l in range(0, 30):
        a = basis.bessel_zeros(l, 60.0)
        b = basis.bessel_zeros(l + 1, 60.0)
        n = min(len(a) - 1, len(b))
        assert np.all(a[:n] < b[:n]) and np.all(b[:n] < a[1:n + 1])


def test_norm_const_radial_orthonormal():
    # c^2 int_0^1 j_l(lam_k r) j_l(lam_k' r) r^2 dr = delta_kk'  (Lommel).
    x, w = np.polynomial.legendre.leggauss(200)
    r = (x + 1) / 2
    w = w / 2 * r * r
    for l in (0, 3, 10, 25):
        lams = basis.bessel_zeros(l, l + 40.0)[:4]
        cs = [basis.norm_const(l, lam) for lam in lams]
        R = np.array([c * special.spherical_jn(l, lam * r) for c, lam in zip(cs, lams)])
        G = (R * w) @ R.T
        np.testing.assert_allclose(G, np.eye(len(lams)), atol=1e-13)


def _count_pairs_mpmath(L):
    cut = float(mpmath.besseljzero(L + 1.5, 1))
    n_rad, n_coef, max_l = 0, 0, 0
    for l in range(0, L + 2):
        k = 1
        while True:
            z = float(mpmath.besseljzero(l + 0.5, k))
            if z >= cut:
                break
            n_rad += 1
            n_coef += 2 * l + 1
            max_l = max(max_l, l)
            k += 1
    return n_rad, n_coef, max_l


@pytest.mark.parametrize("L", [0, 4, 8, 16, 32])
def test_index_set_counts_brute_force(L):
    idx = basis.IndexSet(L)
    n_rad, n_coef, max_l = _count_pairs_mpmath(L)
    assert len(idx.radial) == n_rad
    assert idx.size == n_coef
    assert max_l == L and idx.l.max() == L
    lam = np.array([e[2] for e in idx.radial])
    assert np.all(np.diff(lam) > 0)              # frequency ordered
    # sub-bands are prefixes
    for Ls in range(0, L):
        p = idx.prefix(Ls)
        assert p == basis.IndexSet(Ls).size
        assert np.all(idx.lam[:p] < basis.band_cutoff(Ls))
        assert np.all(idx.lam[p:] >= basis.band_cutoff(Ls))


def test_sph_harm_closed_forms():
    rng = np.random.default_rng(3)
    th = rng.uniform(0, np.pi, 50)
    ph = rng.uniform(0, 2 * np.pi, 50)
    Y = basis.sph_harm
    np.testing.assert_allclose(Y(0, 0, th, ph), 1 / np.sqrt(4 * np.pi), atol=1e-15)
    np.testing.assert_allclose(Y(1, 0, th, ph), np.sqrt(3 / (4 * np.pi)) * np.cos(th), atol=1e-15)
    # Condon-Shortley phase: Y_1^1 = -sqrt(3/8pi) sin(theta) e^{i phi}
    np.testing.assert_allclose(Y(1, 1, th, ph),
                               -np.sqrt(3 / (8 * np.pi)) * np.sin(th) * np.exp(1j * ph), atol=1e-15)
    np.testing.assert_allclose(Y(2, 2, th, ph),
                               0.25 * np.sqrt(15 / (2 * np.pi)) * np.sin(th) ** 2 * np.exp(2j * ph),
                               atol=1e-15)
    np.testing.assert_allclose(Y(2, -1, th, ph),
                               0.5 * np.sqrt(15 / (2 * np.pi)) * np.sin(th) * np.cos(th) * np.exp(-1j * ph),
                               atol=1e-15)
    for l in range(0, 12):
        Pl = np.polynomial.legendre.Legendre.basis(l)(np.cos(th))
        np.testing.assert_allclose(Y(l, 0, th, ph), np.sqrt((2 * l + 1) / (4 * np.pi)) * Pl, atol=1e-13)
        tot = sum(np.abs(Y(l, m, th, ph)) ** 2 for m in range(-l, l + 1))
        np.testing.assert_allclose(tot, (2 * l + 1) / (4 * np.pi), rtol=1e-12)
        for m in range(1, l + 1):
            np.testing.assert_allclose(Y(l, -m, th, ph), (-1) ** m * np.conj(Y(l, m, th, ph)), atol=1e-14)


def exact_ball_quadrature(nr=60, nt=20, nphi=28):
    """Gauss-Legendre in r (weight r^2) x Gauss-Legendre in cos(theta) x trapezoid in phi."""
    xr, wr = np.polynomial.legendre.leggauss(nr)
    r = (xr + 1) / 2
    wr = wr / 2 * r ** 2
    xt, wt = np.polynomial.legendre.leggauss(nt)
    phi = np.arange(nphi) * 2 * np.pi / nphi
    R, CT, PH = np.meshgrid(r, xt, phi, indexing="ij")
    W = (wr[:, None, None] * wt[None, :, None] * np.full(nphi, 2 * np.pi / nphi)[None, None, :]).ravel()
    ST = np.sqrt(1 - CT ** 2)
    X = np.stack([R * ST * np.cos(PH), R * ST * np.sin(PH), R * CT], -1).reshape(-1, 3)
    return X, W


def test_psi_orthonormal_exact_quadrature():
    idx = basis.IndexSet(6)
    X, W = exact_ball_quadrature()
    P = basis.psi(idx, X)
    G = (P.conj().T * W) @ P
    np.testing.assert_allclose(G, np.eye(idx.size), atol=1e-12)


@pytest.mark.parametrize("N", [8, 17, 32, 64])
def test_ball_voxels_integer_count(N):
    # r < 1  <=>  sum (2 i - (N-1))^2 < N^2 for cell-centred samples.
    i = np.arange(N)
    s = (2 * i - (N - 1)) ** 2
    count = int(np.count_nonzero(s[:, None, None] + s[None, :, None] + s[None, None, :] < N * N))
    _h, _xyz, ball = basis.grid(N)
    assert int(ball.sum()) == count
    # grid is symmetric about the origin
    c = _xyz[:, 0, 0, 0]
    np.testing.assert_allclose(c, -c[::-1], atol=0)
    assert math.isclose(_h, 2.0 / N)
