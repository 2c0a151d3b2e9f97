"""Ball-harmonic expansion of voxel volumes (paper Sec. II-A).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper expands volumes with an external fast transform it does not
describe.  We take the plain voxel midpoint quadrature of the L2(B) inner
product that defines the coefficients of an orthonormal basis:

    a_klm = <f, psi_klm> ~= h^3 * sum_{v : r_v < 1} conj(psi_klm(x_v)) f(x_v)

with h = 2/N the voxel edge.  Everything is FP64.  The sum over voxels is a
library matrix product per (l, k) block; no other reordering.
"""

from __future__ import annotations

import numpy as np
from scipy import special

from .basis import IndexSet, grid, spherical


def expand(vols: np.ndarray, idx: IndexSet) -> np.ndarray:
    """Coefficients of a batch of volumes.

    vols: [B, N, N, N] (or [N, N, N]) real or complex samples on the
    cell-centred grid of ``basis.grid``.  Returns complex128 [B, C] (or [C])
    in the layout of ``IndexSet`` (radial entries in lambda order, m=-l..l).
    """
    single = vols.ndim == 3
    v = np.asarray(vols)[None] if single else np.asarray(vols)
    N = v.shape[-1]
    h, xyz, ball = grid(N)
    r, th, ph = spherical(xyz[ball])
    F = v.reshape(v.shape[0], -1)[:, ball.reshape(-1)].astype(np.complex128)
    out = np.zeros((v.shape[0], idx.size), dtype=np.complex128)
    # Y_l^m at every ball voxel, all l <= L and |m| <= L (SciPy's recurrence);
    # Yall[l, m] with negative m at negative indices.
    Yall = special.sph_harm_y_all(idx.L, idx.L, th, ph)
    # j_l(lambda r) only depends on r, which takes few distinct values on the grid.
    r_unique, r_inverse = np.unique(r, return_inverse=True)
    for (l, _k, lam, c), off in zip(idx.radial, idx.offset):
        rad = (c * special.spherical_jn(l, lam * r_unique))[r_inverse]      # [V]
        Y = Yall[l][np.arange(-l, l + 1)].T                                 # [V, 2l+1]
        basis_conj = np.conj(rad[:, None] * Y)                              # conj(psi)
        out[:, off:off + 2 * l + 1] = (h ** 3) * (F @ basis_conj)
    return out[0] if single else out


def synthesize(coeffs: np.ndarray, idx: IndexSet, xyz: np.ndarray) -> np.ndarray:
    """f(x) = sum_c coeffs_c psi_c(x) at points ``xyz[..., 3]`` (Sec. II-A)."""
    from .basis import psi
    return psi(idx, xyz) @ coeffs


def real_symmetric(coeffs: np.ndarray, idx: IndexSet) -> np.ndarray:
    """Project coefficients onto those of a real function.

    For real f, a_{k,l,-m} = (-1)^m conj(a_klm) (from Y_l^{-m} =
    (-1)^m conj(Y_l^m)).  Returns (a + S a)/2 with S that map.
    """
    out = np.array(coeffs, dtype=np.complex128, copy=True)
    sym = np.empty_like(out)
    for (l, _k, _lam, _c), off in zip(idx.radial, idx.offset):
        blk = out[..., off:off + 2 * l + 1]
        ms = np.arange(-l, l + 1)
        sym[..., off:off + 2 * l + 1] = ((-1.0) ** ms) * np.conj(blk[..., ::-1])
    return 0.5 * (out + sym)


def shift_volume(f: np.ndarray, d) -> np.ndarray:
    """f_s[i, j, k] = f[i + dx, j + dy, k + dz] (zero outside the box): the
    sampled f(x + s) for the voxel shift s = d h (Sec. II-C, shift grid)."""
    N = f.shape[0]
    out = np.zeros_like(f)
    src = [slice(max(0, di), min(N, N + di)) for di in d]
    dst = [slice(max(0, -di), min(N, N - di)) for di in d]
    out[dst[0], dst[1], dst[2]] = f[src[0], src[1], src[2]]
    return out
