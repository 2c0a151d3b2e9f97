"""Wigner matrices, Euler angles and rotation metrics (paper Sec. II-A/II-B).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper uses D^l_{m,m'}(g) for the steerability of the basis and in
Eq. (2) without fixing a convention.  Reading used throughout:

* Euler angles are ZYZ and active: R(alpha, beta, gamma) =
  R_z(alpha) R_y(beta) R_z(gamma), and a rotation acts on functions by
  (R_g f)(x) = f(g^{-1} x).
* D^l_{mn}(alpha, beta, gamma) = exp(-i m alpha) d^l_{mn}(beta) exp(-i n gamma)
  with the small-d matrix d^l(beta) = exp(-i beta J_y) in the |l, m> basis,
  m = -l..l (Sakurai / Varshalovich).  With the harmonics of ``basis`` this
  gives a(R_g f) = D^l(g) a(f) for each radial block.

Small-d is computed here from its definition: J_y is diagonalised once per
degree (Hermitian eigendecomposition) and d^l(beta) = V diag(e^{-i mu beta}) V^H.
The beta-derivative is the exact matrix identity d'(beta) = -i J_y d(beta).
Neither uses a recurrence in l.
"""

from __future__ import annotations

import functools

import numpy as np


# ------------------------------------------------------------- rotations ----

def rot_z(a: float) -> np.ndarray:
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_y(b: float) -> np.ndarray:
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def euler_to_matrix(alpha: float, beta: float, gamma: float) -> np.ndarray:
    """R(alpha, beta, gamma) = R_z(alpha) R_y(beta) R_z(gamma)."""
    return rot_z(alpha) @ rot_y(beta) @ rot_z(gamma)


def matrix_to_euler(R: np.ndarray) -> np.ndarray:
    """Inverse of ``euler_to_matrix``; beta in [0, pi], alpha, gamma in (-pi, pi]."""
    R = np.asarray(R, dtype=np.float64)
    beta = float(np.arccos(np.clip(R[2, 2], -1.0, 1.0)))
    sb = np.hypot(R[0, 2], R[1, 2])
    if sb > 1e-12:
        alpha = float(np.arctan2(R[1, 2], R[0, 2]))
        gamma = float(np.arctan2(R[2, 1], -R[2, 0]))
    else:  # gimbal lock: only alpha +/- gamma is defined; put it in alpha
        gamma = 0.0
        alpha = float(np.arctan2(R[1, 0], R[0, 0]))
        if R[2, 2] < 0:
            alpha = float(np.arctan2(-R[1, 0], -R[0, 0]))
    return np.array([alpha, beta, gamma])


def geodesic_deg(Ra: np.ndarray, Rb: np.ndarray) -> float:
    """Angle (degrees) of the rotation Ra Rb^T, from the Frobenius distance.

    ||Ra - Rb||_F = 2 sqrt(2) sin(theta / 2) for a relative rotation by theta.
    """
    d = np.linalg.norm(np.asarray(Ra) - np.asarray(Rb))
    return float(np.degrees(2.0 * np.arcsin(min(1.0, d / (2.0 * np.sqrt(2.0))))))


# ----------------------------------------------------------------- small d ----

@functools.lru_cache(maxsize=None)
def _jy_eig(l: int):
    """Eigen-decomposition of J_y for degree l (basis m = -l..l)."""
    n = 2 * l + 1
    jp = np.zeros((n, n))
    for i, m in enumerate(range(-l, l)):          # J_+ |m> = sqrt((l-m)(l+m+1)) |m+1>
        jp[i + 1, i] = np.sqrt((l - m) * (l + m + 1.0))
    jy = (jp - jp.T) / 2j                          # J_y = (J_+ - J_-)/(2i)
    mu, V = np.linalg.eigh(jy)
    return jy, mu, V


def jy_matrix(l: int) -> np.ndarray:
    return _jy_eig(l)[0]


def small_d(l: int, beta) -> np.ndarray:
    """d^l(beta) = exp(-i beta J_y); rows/cols m = -l..l.

    ``beta`` scalar -> [2l+1, 2l+1]; array [P] -> [P, 2l+1, 2l+1].
    """
    _jy, mu, V = _jy_eig(l)
    b = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    ph = np.exp(-1j * mu[None, :] * b[:, None])             # [P, n]
    d = np.einsum("ij,pj,kj->pik", V, ph, V.conj()).real
    return d[0] if np.ndim(beta) == 0 else d


def small_d_prime(l: int, beta) -> np.ndarray:
    """d/dbeta d^l(beta) = -i J_y d^l(beta) (exact matrix identity)."""
    jy = jy_matrix(l)
    d = small_d(l, beta)
    return np.real(np.matmul(-1j * jy, d))


def small_d_second(l: int, beta) -> np.ndarray:
    """d^2/dbeta^2 d^l(beta) = -J_y^2 d^l(beta) (exact matrix identity)."""
    jy = jy_matrix(l)
    d = small_d(l, beta)
    return np.real(np.matmul(-(jy @ jy), d))


def wigner_D(l: int, alpha: float, beta: float, gamma: float) -> np.ndarray:
    """D^l_{mn}(alpha, beta, gamma) = e^{-i m alpha} d^l_{mn}(beta) e^{-i n gamma}."""
    m = np.arange(-l, l + 1)
    return (np.exp(-1j * m * alpha)[:, None] * small_d(l, beta)
            * np.exp(-1j * m * gamma)[None, :])


# ------------------------------------------------------------- Euler wrap ----

def wrap_angle(t: float) -> float:
    """Map an angle to [-pi, pi)."""
    return t - 2.0 * np.pi * np.floor((t + np.pi) / (2.0 * np.pi))


def wrap_euler(e) -> np.ndarray:
    """Canonical ZYZ triple: beta in [0, pi], alpha, gamma in [-pi, pi).

    Uses R(alpha, beta, gamma) = R(alpha + pi, 2 pi - beta, gamma + pi), which
    follows from R_z(pi) R_y(b) R_z(-pi) = R_y(-b).
    """
    a, b, g = (float(x) for x in e)
    b = b - 2.0 * np.pi * np.floor(b / (2.0 * np.pi))        # [0, 2pi)
    if b > np.pi:
        b = 2.0 * np.pi - b
        a += np.pi
        g += np.pi
    return np.array([wrap_angle(a), b, wrap_angle(g)])
