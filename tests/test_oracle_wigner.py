"""Pins of the oracle's Wigner matrices and Euler conventions.

d^l against Wigner's explicit factorial sum (mpmath, independent of the
J_y eigendecomposition), the l = 1 closed forms and d^l_00 = P_l(cos b);
D^l against unitarity and the group law D(g1 g2) = D(g1) D(g2) with the
product taken on rotation matrices; d' against central differences; Euler
conversions and the wrap rule against rotation matrices.
"""

import mpmath
import numpy as np
import pytest

from oracle import wigner


def wigner_d_factorial(l, m, n, beta):
    """Wigner's formula for d^l_{mn}(beta) in exact arithmetic (mpmath)."""
    mpmath.mp.dps = 40
    b = mpmath.mpf(beta)
    c, s = mpmath.cos(b / 2), mpmath.sin(b / 2)
    f = mpmath.factorial
    pref = mpmath.sqrt(f(l + m) * f(l - m) * f(l + n) * f(l - n))
    tot = mpmath.mpf(0)
    for k in range(0, 2 * l + 1):
        a1, a2, a3, a4 = l + n - k, k, m - n + k, l - m - k
        if min(a1, a2, a3, a4) < 0:
            continue
        tot += ((-1) ** (m - n + k) * c ** (2 * l + n - m - 2 * k) * s ** (m - n + 2 * k)
                / (f(a1) * f(a2) * f(a3) * f(a4)))
    return float(pref * tot)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 6, 10])
def test_small_d_factorial_sum(l):
    for beta in (0.0, 0.3, 1.2, np.pi / 2, 2.5, np.pi):
        d = wigner.small_d(l, beta)
        for i, m in enumerate(range(-l, l + 1)):
            for j, n in enumerate(range(-l, l + 1)):
                assert abs(d[i, j] - wigner_d_factorial(l, m, n, beta)) < 1e-13


def test_small_d_l1_closed_forms():
    for b in np.linspace(0, np.pi, 7):
        d = wigner.small_d(1, b)          # rows/cols m = -1, 0, 1
        c, s = np.cos(b), np.sin(b)
        ref = np.array([[(1 + c) / 2, s / np.sqrt(2), (1 - c) / 2],
                        [-s / np.sqrt(2), c, s / np.sqrt(2)],
                        [(1 - c) / 2, -s / np.sqrt(2), (1 + c) / 2]])
        np.testing.assert_allclose(d, ref, atol=1e-15)


def test_small_d_00_is_legendre():
    for l in range(0, 20):
        for b in (0.1, 0.9, 2.0, 3.0):
            ref = np.polynomial.legendre.Legendre.basis(l)(np.cos(b))
            assert abs(wigner.small_d(l, b)[l, l] - ref) < 1e-13


def test_small_d_symmetries():
    for l in (3, 8):
        ms = np.arange(-l, l + 1)
        sign = (-1.0) ** (ms[:, None] - ms[None, :])
        for b in (0.4, 1.9):
            d = wigner.small_d(l, b)
            np.testing.assert_allclose(d.T, sign * d, atol=1e-14)           # d_nm = (-1)^{m-n} d_mn
            np.testing.assert_allclose(d[::-1, ::-1], sign * d, atol=1e-14)  # d_{-m,-n}


def test_small_d_prime_finite_difference():
    for l in (1, 5, 12):
        for b in (0.2, 1.3, 2.9):
            h = 1e-5
            fd = (wigner.small_d(l, b + h) - wigner.small_d(l, b - h)) / (2 * h)
            np.testing.assert_allclose(wigner.small_d_prime(l, b), fd, atol=1e-9)


def test_D_unitary_and_group_law():
    rng = np.random.default_rng(5)
    for _ in range(4):
        e1 = np.array([rng.uniform(-np.pi, np.pi), rng.uniform(0, np.pi), rng.uniform(-np.pi, np.pi)])
        e2 = np.array([rng.uniform(-np.pi, np.pi), rng.uniform(0, np.pi), rng.uniform(-np.pi, np.pi)])
        R12 = wigner.euler_to_matrix(*e1) @ wigner.euler_to_matrix(*e2)
        e12 = wigner.matrix_to_euler(R12)
        Rinv = wigner.euler_to_matrix(*e1).T
        einv = wigner.matrix_to_euler(Rinv)
        for l in (1, 4, 9):
            D1 = wigner.wigner_D(l, *e1)
            D2 = wigner.wigner_D(l, *e2)
            np.testing.assert_allclose(D1 @ D1.conj().T, np.eye(2 * l + 1), atol=1e-13)
            np.testing.assert_allclose(wigner.wigner_D(l, *e12), D1 @ D2, atol=1e-13)
            np.testing.assert_allclose(wigner.wigner_D(l, *einv), D1.conj().T, atol=1e-13)


def test_D_l1_matches_rotation_matrix():
    # The linear function x -> v.x has degree-1 coefficients proportional to
    # <Y_1^m, v.x/r> = U v with rows conj(Y_1^m) in Cartesian form
    # (Y_1^{+1} ~ -(x + i y)/sqrt2, Y_1^0 ~ z, Y_1^{-1} ~ (x - i y)/sqrt2).
    # Rotating the function by g maps v -> g v, so D^1(g) = U g U^H.
    U = np.array([[1 / np.sqrt(2), 1j / np.sqrt(2), 0],       # m = -1
                  [0, 0, 1],                                   # m = 0
                  [-1 / np.sqrt(2), 1j / np.sqrt(2), 0]])      # m = +1
    rng = np.random.default_rng(9)
    for _ in range(5):
        e = np.array([rng.uniform(-np.pi, np.pi), rng.uniform(0, np.pi), rng.uniform(-np.pi, np.pi)])
        R = wigner.euler_to_matrix(*e)
        np.testing.assert_allclose(wigner.wigner_D(1, *e), U @ R @ U.conj().T, atol=1e-14)


def test_euler_roundtrip_and_wrap():
    rng = np.random.default_rng(11)
    for _ in range(50):
        e = rng.uniform(-7, 7, 3)
        R = wigner.euler_to_matrix(*e)
        w = wigner.wrap_euler(e)
        assert 0 <= w[1] <= np.pi and -np.pi <= w[0] < np.pi and -np.pi <= w[2] < np.pi
        np.testing.assert_allclose(wigner.euler_to_matrix(*w), R, atol=1e-13)
        e2 = wigner.matrix_to_euler(R)
        np.testing.assert_allclose(wigner.euler_to_matrix(*e2), R, atol=1e-12)


def test_geodesic_angle():
    rng = np.random.default_rng(2)
    for th in (0.0, 1e-4, 0.3, 1.5, 3.0):
        ax = rng.standard_normal(3)
        ax /= np.linalg.norm(ax)
        K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        Rrel = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K   # Rodrigues
        Rb = wigner.euler_to_matrix(0.3, 1.1, -0.7)
        assert abs(wigner.geodesic_deg(Rrel @ Rb, Rb) - np.degrees(th)) < 1e-9
