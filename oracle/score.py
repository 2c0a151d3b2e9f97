"""Rotational cross-correlation in the ball-harmonic domain (paper Eq. (2)).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Eq. (1) at zero shift, for band-limited t (coefficients b) and f
(coefficients a), is

    C(g) = int t(x) [R_g f](x) dx = sum_{klm} conj(b_klm) [D(g) a]_klm
         = sum_l sum_{m,n} xi^l_{mn} D^l_{mn}(g),                 (Eq. (2))

    xi^l_{mn} = sum_{k in band} conj(b_klm) a_kln.

So the coefficients xi^s of Eq. (2) (zero shift) are the per-degree
cross-power matrices between template and particle.  For real t and f the
sum is real; we return its real part.  Euler gradient (closed form, Sec. II-C):
d/dalpha brings -i m, d/dgamma brings -i n, d/dbeta replaces d^l by its
derivative.
"""

from __future__ import annotations

import numpy as np

from .basis import IndexSet, band_cutoff
from . import wigner


def band_mask(idx: IndexSet, L: int) -> np.ndarray:
    """Coefficients of band L: lambda_lk < lambda_{L+1,1} (a prefix)."""
    return idx.lam < band_cutoff(L)


def cross_power(a: np.ndarray, b: np.ndarray, idx: IndexSet, L: int):
    """xi^l for l = 0..L: list of complex [2l+1, 2l+1] matrices.

    a: particle coefficients [C]; b: template coefficients [C] (same index set).
    """
    keep = band_mask(idx, L)
    xi = [np.zeros((2 * l + 1, 2 * l + 1), dtype=np.complex128) for l in range(L + 1)]
    for (l, _k, lam, _c), off in zip(idx.radial, idx.offset):
        if not keep[off]:
            continue
        bl = b[off:off + 2 * l + 1]
        al = a[off:off + 2 * l + 1]
        xi[l] += np.outer(np.conj(bl), al)
    return xi


def score_grad(xi, euler):
    """S and dS/d(alpha, beta, gamma) at Euler triples.

    euler: [P, 3].  Returns (S [P], grad [P, 3]) in FP64.
    """
    e = np.atleast_2d(np.asarray(euler, dtype=np.float64))
    P = e.shape[0]
    S = np.zeros(P)
    G = np.zeros((P, 3))
    al, be, ga = e[:, 0], e[:, 1], e[:, 2]
    for l, x in enumerate(xi):
        if not np.any(x):
            continue
        m = np.arange(-l, l + 1)
        d = wigner.small_d(l, be).reshape(P, 2 * l + 1, 2 * l + 1)
        dp = wigner.small_d_prime(l, be).reshape(P, 2 * l + 1, 2 * l + 1)
        pa = np.exp(-1j * m[None, :] * al[:, None])            # [P, m]
        pg = np.exp(-1j * m[None, :] * ga[:, None])            # [P, n]
        W = x[None] * pa[:, :, None] * pg[:, None, :]          # xi e^{-i m a} e^{-i n g}
        S += np.real(np.sum(W * d, axis=(1, 2)))
        G[:, 0] += np.real(np.sum(W * d * (-1j * m)[None, :, None], axis=(1, 2)))
        G[:, 1] += np.real(np.sum(W * dp, axis=(1, 2)))
        G[:, 2] += np.real(np.sum(W * d * (-1j * m)[None, None, :], axis=(1, 2)))
    return S, G


def score(xi, euler):
    return score_grad(xi, euler)[0]


def score_grad_hess(xi, euler):
    """S, gradient and Hessian in (alpha, beta, gamma) at Euler triples.

    Second derivatives of D^l_{mn} = e^{-i m alpha} d^l_{mn}(beta) e^{-i n gamma}:
    alpha brings -i m, gamma brings -i n, beta replaces d by d' or d''.
    Returns (S [P], grad [P, 3], hess [P, 3, 3]).
    """
    e = np.atleast_2d(np.asarray(euler, dtype=np.float64))
    P = e.shape[0]
    S = np.zeros(P)
    G = np.zeros((P, 3))
    H = np.zeros((P, 3, 3))
    al, be, ga = e[:, 0], e[:, 1], e[:, 2]
    for l, x in enumerate(xi):
        if not np.any(x):
            continue
        m = np.arange(-l, l + 1)
        d = wigner.small_d(l, be).reshape(P, 2 * l + 1, 2 * l + 1)
        d1 = wigner.small_d_prime(l, be).reshape(P, 2 * l + 1, 2 * l + 1)
        d2 = wigner.small_d_second(l, be).reshape(P, 2 * l + 1, 2 * l + 1)
        pa = np.exp(-1j * m[None, :] * al[:, None])
        pg = np.exp(-1j * m[None, :] * ga[:, None])
        W = x[None] * pa[:, :, None] * pg[:, None, :]
        fa = (-1j * m)[None, :, None]          # d/dalpha on D_{mn}
        fg = (-1j * m)[None, None, :]          # d/dgamma on D_{mn}
        re = lambda t: np.real(np.sum(t, axis=(1, 2)))
        S += re(W * d)
        G[:, 0] += re(W * d * fa)
        G[:, 1] += re(W * d1)
        G[:, 2] += re(W * d * fg)
        H[:, 0, 0] += re(W * d * fa * fa)
        H[:, 0, 1] += re(W * d1 * fa)
        H[:, 0, 2] += re(W * d * fa * fg)
        H[:, 1, 1] += re(W * d2)
        H[:, 1, 2] += re(W * d1 * fg)
        H[:, 2, 2] += re(W * d * fg * fg)
    H[:, 1, 0] = H[:, 0, 1]
    H[:, 2, 0] = H[:, 0, 2]
    H[:, 2, 1] = H[:, 1, 2]
    return S, G, H


def degree_energy(a: np.ndarray, b: np.ndarray, idx: IndexSet, L: int) -> np.ndarray:
    """||xi^l||_F^2 for l = 0..L: energy of each degree of the band-L cross-power."""
    return np.array([float(np.sum(np.abs(x) ** 2)) for x in cross_power(a, b, idx, L)])


def energy_ratio(energy: np.ndarray) -> np.ndarray:
    """Ratio(L) = sum_{l > L} E_l / sum_l E_l for L = 0..len(E)-1 (the energy
    of the degrees a truncation at L leaves out, as a fraction of all)."""
    E = np.asarray(energy, dtype=np.float64)
    tot = E.sum()
    tail = tot - np.cumsum(E)
    return tail / tot if tot > 0 else np.zeros_like(E)


def select_bands(ratio: np.ndarray, thresholds) -> list:
    """For each threshold tau (any order), the smallest L with Ratio(L) <= tau;
    the distinct values in increasing order."""
    r = np.asarray(ratio)
    out = set()
    for tau in thresholds:
        hit = np.nonzero(r <= tau)[0]
        out.add(int(hit[0]) if hit.size else len(r) - 1)
    return sorted(out)


def select_bands_batch(ratios: np.ndarray, thresholds) -> list:
    """The batch's band for each threshold tau (in the order given): the
    smallest L with Ratio_b(L) <= tau for at least ceil(B/2) of the B
    particles' ratio curves ``ratios[b]`` (the paper picks one band set for
    a data set, Sec. III; half of the particles is the reading taken for
    "the data set").  Counted by brute force over L and b."""
    r = np.asarray(ratios, dtype=np.float64)
    B, n = r.shape
    need = (B + 1) // 2
    out = []
    for tau in thresholds:
        pick = n - 1
        for L in range(n):
            if sum(1 for b in range(B) if r[b, L] <= tau) >= need:
                pick = L
                break
        out.append(pick)
    return out


def band_norms(a: np.ndarray, b: np.ndarray, idx: IndexSet, L: int):
    """Per-degree norms ||a_l||, ||b_l|| over band L (l = 0..L)."""
    keep = band_mask(idx, L)
    na = np.zeros(L + 1)
    nb = np.zeros(L + 1)
    for l in range(L + 1):
        sel = keep & (idx.l == l)
        na[l] = np.sqrt(np.sum(np.abs(a[sel]) ** 2))
        nb[l] = np.sqrt(np.sum(np.abs(b[sel]) ** 2))
    return na, nb


def cs_bound(a, b, idx, L) -> float:
    """Cauchy-Schwarz bound of |C(g)| over band L: ||a||_band ||b||_band."""
    keep = band_mask(idx, L)
    return float(np.linalg.norm(a[keep]) * np.linalg.norm(b[keep]))


def curvature_weight(a, b, idx, L) -> float:
    """W_L = sum_{l<=L} l(l+1) ||a_l|| ||b_l||.

    Bound on |sum_l l(l+1) C_l(g)|, the magnitude of the SO(3) Laplacian of
    the band-L score (Delta D^l = -l(l+1) D^l); used to scale the first
    ascent step of each band.
    """
    na, nb = band_norms(a, b, idx, L)
    ll = np.arange(L + 1)
    return float(np.sum(ll * (ll + 1) * na * nb))
