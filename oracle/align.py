"""Frequency marching with multi-start gradient ascent (paper Sec. II-C).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper maximises Eq. (2) by truncating the degree sum at a bandlimit L
that is raised band by band (frequency marching) and by following the
closed-form gradient instead of sampling SO(3) exhaustively.  It gives no
step rule; the rule used on both sides of the parity tests is:

1. Starts: P rotations as ZYZ Euler triples (drawn by the caller).
2. For each band L_b in the schedule, with the band's cross-power xi:
   evaluate (S, grad S) at the carried point x; set the step
   eta = step_init / W_b (W_b from ``score.curvature_weight``; 0 if W_b = 0).
   Then T times: x' = wrap(x + eta * grad S(x)); evaluate at x'.  If
   S(x') >= S(x) accept (x <- x', with its score and gradient) and
   eta <- eta * grow; otherwise keep x and eta <- eta * shrink.
3. After the last band the restart of highest score wins (lowest index on
   ties).

All arithmetic is FP64.
"""

from __future__ import annotations

import numpy as np

from .basis import IndexSet
from . import score as sc
from . import wigner


def wrap_many(x: np.ndarray) -> np.ndarray:
    return np.stack([wigner.wrap_euler(e) for e in x]) if len(x) else x.copy()


def ascent_direction(x: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Riemannian (natural) gradient in ZYZ Euler coordinates: g^{-1} grad S.

    The bi-invariant metric of SO(3) in ZYZ coordinates is
    [[1, 0, cos b], [0, 1, 0], [cos b, 0, 1]]; its inverse is applied to the
    Euler gradient.  The metric is singular where sin b = 0, so sin^2 b is
    floored at ``SIN2_FLOOR``.
    """
    c = np.cos(x[:, 1])
    s2 = np.maximum(1.0 - c * c, SIN2_FLOOR)
    da = (G[:, 0] - c * G[:, 2]) / s2
    dg = (G[:, 2] - c * G[:, 0]) / s2
    return np.stack([da, G[:, 1], dg], axis=1)


SIN2_FLOOR = 1e-6


def march(a, b, idx: IndexSet, bands, starts, steps: int,
          step_init: float = 1.0, grow: float = 1.25, shrink: float = 0.5,
          trace: bool = False):
    """Run the ascent for one particle.

    a, b: particle / template coefficients [C] (complex).
    starts: [P, 3] Euler triples.  Returns dict with ``euler`` [P, 3],
    ``score`` [P], ``best`` (index), and ``trace`` (list of per-band
    [T+1, P] score arrays) if requested.
    """
    x = wrap_many(np.asarray(starts, dtype=np.float64))
    P = x.shape[0]
    S = np.full(P, -np.inf)
    hist = []
    for L in bands:
        xi = sc.cross_power(a, b, idx, L)
        W = sc.curvature_weight(a, b, idx, L)
        eta = np.full(P, step_init / W if W > 0 else 0.0)
        S, G = sc.score_grad(xi, x)
        band_hist = [S.copy()]
        for _ in range(steps):
            xt = wrap_many(x + eta[:, None] * ascent_direction(x, G))
            St, Gt = sc.score_grad(xi, xt)
            acc = St >= S
            x[acc] = xt[acc]
            S = np.where(acc, St, S)
            G[acc] = Gt[acc]
            eta = np.where(acc, eta * grow, eta * shrink)
            band_hist.append(S.copy())
        hist.append(np.array(band_hist))
    best = int(np.argmax(S)) if P else -1
    out = {"euler": x, "score": S, "best": best}
    if trace:
        out["trace"] = hist
    return out


def align_batch(A, b, idx: IndexSet, bands, starts, steps: int, **kw):
    """Best rotation per particle: (euler [B, 3], score [B]).

    A: [B, C] particle coefficients; starts: [B, P, 3].
    """
    eu = np.zeros((A.shape[0], 3))
    s = np.zeros(A.shape[0])
    for i in range(A.shape[0]):
        r = march(A[i], b, idx, bands, starts[i], steps, **kw)
        eu[i] = r["euler"][r["best"]]
        s[i] = r["score"][r["best"]]
    return eu, s
