"""The mirror-fold rewrite of the voxel quadrature (paper Sec. II-A) on the CPU.

The library sums the expansion over one voxel per orbit of the three
coordinate reflections.  This test restates that rewrite in NumPy and checks
it against the oracle's dense voxel sum, so the regrouping is pinned without
the GPU:

* The cell-centred ball is invariant under x -> -x, y -> -y, z -> -z.
* Each real basis column has a definite sign under each reflection.  For
  conj(psi_klm) = c_lk j_l(lam r) N_lm P_l^m(cos t) e^{-i m p}, m >= 0:
  the real part (cos m p) is even in y and has sign (-1)^m under x -> -x;
  the imaginary part (-sin m p) is odd in y and has sign (-1)^(m+1) under
  x -> -x; both have sign (-1)^(l+m) under z -> -z (P_l^m(-u) =
  (-1)^(l+m) P_l^m(u)); the radial factor is even.
* So sum_v f(v) psi(v) = sum_{v >= 0} psi(v) g_P(v) / |stab(v)|, with
  g_P(v) = sum over the 8 reflections R of chi_P(R) f(R v) (chi_P(R) the
  product of the column's signs over the axes R flips), and |stab(v)| =
  2^(number of zero coordinates of v) on odd grids (1 on even grids).
* The representatives are the voxels with x, y, z >= 0.

A wrong parity bit, a missing stabiliser weight or a wrong set of
representatives changes the sum by O(1) relative, far above the 1e-13 bar.
"""

import numpy as np
import pytest

from oracle import basis, expand


def folded_expand(f, idx):
    """Real columns (Re, Im of conj psi, m >= 0) summed over representatives."""
    N = f.shape[0]
    h, xyz, ball = basis.grid(N)
    c = xyz[:, 0, 0, 0]
    rep = np.nonzero(c >= -1e-12)[0]                 # coordinate >= 0 on each axis
    sub = np.ix_(rep, rep, rep)
    flip = lambda a, ax: np.flip(a, axis=ax)
    # images f(R v) at the representatives for each reflection (sx, sy, sz)
    images = {}
    for sx in (0, 1):
        for sy in (0, 1):
            for sz in (0, 1):
                g = f
                if sx: g = flip(g, 0)
                if sy: g = flip(g, 1)
                if sz: g = flip(g, 2)
                images[(sx, sy, sz)] = g[sub]
    zero = np.abs(c[rep]) < 1e-12
    nz = zero[:, None, None].astype(int) + zero[None, :, None] + zero[None, None, :]
    weight = ball[sub] / (2.0 ** nz)
    psi_rep = basis.psi(idx, xyz[sub])              # [n, n, n, C]
    out = np.zeros(idx.size, dtype=np.complex128)
    for (l, _k, _lam, _c), off in zip(idx.radial, idx.offset):
        for m in range(0, l + 1):
            col = np.conj(psi_rep[..., off + l + m])
            for part, px, py in ((0, (-1) ** m, 1), (1, (-1) ** (m + 1), -1)):
                pz = (-1) ** (l + m)
                gP = sum(images[s] * (px if s[0] else 1) * (py if s[1] else 1) * (pz if s[2] else 1)
                         for s in images)
                basis_col = col.real if part == 0 else col.imag
                val = h ** 3 * np.sum(basis_col * gP * weight)
                if part == 0:
                    out[off + l + m] += val
                else:
                    out[off + l + m] += 1j * val
    # m < 0 from real-input symmetry: a_{k,l,-m} = (-1)^m conj(a_klm)
    for (l, _k, _lam, _c), off in zip(idx.radial, idx.offset):
        for m in range(1, l + 1):
            out[off + l - m] = (-1) ** m * np.conj(out[off + l + m])
    return out


@pytest.mark.parametrize("N", [9, 10, 17])
def test_fold_equals_dense_voxel_sum(N):
    idx = basis.IndexSet(5)
    rng = np.random.default_rng(N)
    f = rng.standard_normal((N, N, N))
    dense = expand.expand(f, idx)
    folded = folded_expand(f, idx)
    assert np.linalg.norm(folded - dense) <= 1e-13 * np.linalg.norm(dense)
