"""Ball-harmonic basis (paper Sec. II-A, the unnumbered basis equation).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

psi_klm(r, theta, phi) = c_lk * j_l(lambda_lk r) * Y_l^m(theta, phi) * 1[r < 1]

* lambda_lk is the k-th positive zero of the spherical Bessel function j_l.
* c_lk is a positive normalisation constant.  The paper does not give its
  value; we take the one that makes psi_klm orthonormal in L2(B):
  c_lk = sqrt(2) / |j_{l+1}(lambda_lk)|  (Lommel's integral at a zero of j_l).
* Y_l^m is the complex, orthonormal spherical harmonic with the
  Condon-Shortley phase, theta polar from +z, phi azimuth from +x
  (SciPy's ``sph_harm_y``).
* Frequency order: basis functions are sorted by their Dirichlet-Laplacian
  eigenvalue lambda_lk^2 (Sec. II-A, "frequency-ordered").  The band of
  bandlimit L is read as the isotropic low-pass
  I(L) = {(k, l, m) : lambda_lk < lambda_{L+1,1}}, a prefix of that order
  (so l <= L holds automatically).  Ties in lambda are broken by (l, k).

Grid convention: an N^3 box covers [-1, 1]^3 with cell-centred samples
x_i = (i - (N-1)/2) * h, h = 2/N; ``vol[i, j, k]`` is the sample at
(x_i, y_j, z_k).  Only voxels with r < 1 enter (the indicator in psi).
"""

from __future__ import annotations

import numpy as np
from scipy import optimize, special


# ---------------------------------------------------------------- zeros ----

def bessel_zeros(l: int, x_max: float) -> np.ndarray:
    """All positive zeros of j_l below ``x_max``, ascending, to ~1e-15.

    Zeros are bracketed by sign changes on a 0.05-spaced grid (consecutive
    zeros of j_l are more than pi apart) and refined with Brent's method.
    """
    if x_max <= 0:
        return np.zeros(0)
    # j_l has no zero in (0, l]; start the scan just above l (or at 0.05).
    x = np.arange(max(float(l), 0.05), x_max + 0.05, 0.05)
    y = special.spherical_jn(l, x)
    out = []
    for i in range(len(x) - 1):
        if y[i] == 0.0:
            out.append(x[i])
        elif y[i] * y[i + 1] < 0:
            out.append(optimize.brentq(lambda t: special.spherical_jn(l, t),
                                       x[i], x[i + 1], xtol=1e-15, rtol=8.9e-16,
                                       maxiter=200))
    return np.array([z for z in out if z < x_max])


def first_zero(l: int) -> float:
    """lambda_{l,1}: the first positive zero of j_l."""
    z = bessel_zeros(l, l + 2.0 * np.pi + 4.0)
    return float(z[0])


def band_cutoff(L: int) -> float:
    """Cut-off eigen-frequency of band L: lambda_{L+1,1} (reading of Sec. II-A)."""
    return first_zero(L + 1)


def norm_const(l: int, lam: float) -> float:
    """c_lk = sqrt(2)/|j_{l+1}(lambda_lk)| -- L2(B) normalisation of psi."""
    return float(np.sqrt(2.0) / abs(special.spherical_jn(l + 1, lam)))


# ------------------------------------------------------------ index set ----

class IndexSet:
    """Frequency-ordered index set I(L) and its complex-coefficient layout.

    ``radial``: list of (l, k, lambda_lk, c_lk) in ascending lambda.
    Coefficient layout: for each radial entry in that order, m = -l..l.
    ``l, k, m, lam``: per-coefficient arrays of length C(L).
    """

    def __init__(self, L: int):
        self.L = int(L)
        cut = band_cutoff(self.L)
        rad = []
        for l in range(0, self.L + 1):
            for kk, lam in enumerate(bessel_zeros(l, cut), start=1):
                if lam < cut:
                    rad.append((l, kk, float(lam)))
        rad.sort(key=lambda t: (t[2], t[0], t[1]))
        self.cutoff = cut
        self.radial = [(l, k, lam, norm_const(l, lam)) for (l, k, lam) in rad]
        ls, ks, ms, lams = [], [], [], []
        self.offset = []          # first coefficient index of each radial entry
        for (l, k, lam, _c) in self.radial:
            self.offset.append(len(ls))
            for m in range(-l, l + 1):
                ls.append(l); ks.append(k); ms.append(m); lams.append(lam)
        self.l = np.array(ls, dtype=np.int64)
        self.k = np.array(ks, dtype=np.int64)
        self.m = np.array(ms, dtype=np.int64)
        self.lam = np.array(lams, dtype=np.float64)

    @property
    def size(self) -> int:
        """C(L): number of complex coefficients (all m)."""
        return int(self.l.size)

    def prefix(self, L: int) -> int:
        """Number of coefficients of the sub-band L <= self.L (a prefix)."""
        cut = band_cutoff(L)
        return int(np.count_nonzero(self.lam < cut))


# ----------------------------------------------------------------- grid ----

def grid(N: int):
    """Cell-centred grid on [-1,1]^3.

    Returns (h, xyz[N,N,N,3], ball_mask[N,N,N]) with ball = r < 1.
    """
    h = 2.0 / N
    c = (np.arange(N) - (N - 1) / 2.0) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    xyz = np.stack([X, Y, Z], axis=-1)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    return h, xyz, r < 1.0


def spherical(xyz: np.ndarray):
    """(r, theta, phi) of Cartesian points; theta polar from +z, phi in [0, 2pi)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    safe = np.where(r > 0, r, 1.0)
    theta = np.arccos(np.clip(np.where(r > 0, z / safe, 1.0), -1.0, 1.0))
    phi = np.mod(np.arctan2(y, x), 2.0 * np.pi)
    return r, theta, phi


# ---------------------------------------------------------- evaluation ----

def sph_harm(l: int, m: int, theta, phi):
    """Complex orthonormal Y_l^m with Condon-Shortley phase."""
    return special.sph_harm_y(l, m, theta, phi)


def psi(idx: IndexSet, xyz: np.ndarray) -> np.ndarray:
    """All basis functions of ``idx`` at points ``xyz[..., 3]``.

    Returns complex array [..., C] with psi_klm(x) (zero where r >= 1).
    """
    r, th, ph = spherical(xyz)
    inside = r < 1.0
    out = np.zeros(r.shape + (idx.size,), dtype=np.complex128)
    for (l, k, lam, c), off in zip(idx.radial, idx.offset):
        rad = c * special.spherical_jn(l, lam * r) * inside
        for j, m in enumerate(range(-l, l + 1)):
            out[..., off + j] = rad * sph_harm(l, m, th, ph)
    return out
