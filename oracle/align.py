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

Optional refinements of the paper's own procedure (Newton steps on
candidate rotations, candidates from the local maxima of the lowest band)
are described in ``march``.

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


NEWTON_MAX_STEP = 0.5


def newton_direction(x: np.ndarray, G: np.ndarray, H: np.ndarray, eta0: float) -> np.ndarray:
    """Step of a Newton band for each restart.

    Where -H is positive definite (its three leading principal minors are
    positive) the Newton step -H^{-1} grad S towards the stationary point of
    the local quadratic model; elsewhere the natural-gradient step
    eta0 * g^{-1} grad S of the gradient bands.  Either is scaled down to a
    largest component of NEWTON_MAX_STEP radians.
    """
    nat = eta0 * ascent_direction(x, G)
    d = np.empty_like(nat)
    for i in range(len(x)):
        Hn = -H[i]
        m1 = Hn[0, 0]
        m2 = Hn[0, 0] * Hn[1, 1] - Hn[0, 1] * Hn[1, 0]
        m3 = np.linalg.det(Hn)
        if m1 > 0 and m2 > 0 and m3 > 0:
            d[i] = np.linalg.solve(Hn, G[i])
        else:
            d[i] = nat[i]
        big = np.max(np.abs(d[i]))
        if big > NEWTON_MAX_STEP:
            d[i] *= NEWTON_MAX_STEP / big
    return d


def prune_candidates(x: np.ndarray, S: np.ndarray, keep: int, min_sep: float) -> np.ndarray:
    """Indices of `keep` candidate restarts: distinct local maxima first.

    Restarts are visited by decreasing score (lower index first on ties); one
    is taken if its rotation is more than `min_sep` radians from every one
    taken so far (angle t between rotations: 3 - tr(Ra^T Rb) = 4 sin^2(t/2)),
    until `keep` are taken.  If fewer are distinct, the remaining slots are
    filled with the skipped restarts in the same order.
    """
    order = sorted(range(len(S)), key=lambda i: (-S[i], i))
    R = [wigner.euler_to_matrix(*e) for e in x]
    thr = 4.0 * np.sin(0.5 * min_sep) ** 2
    chosen = []
    for i in order:
        if len(chosen) == keep:
            break
        if all(3.0 - np.trace(R[i].T @ R[j]) > thr for j in chosen):
            chosen.append(i)
    if len(chosen) < keep:
        rest = [i for i in order if i not in chosen]
        chosen += rest[:keep - len(chosen)]
    return np.array(chosen, dtype=np.int64)


def march(a, b, idx: IndexSet, bands, starts, steps: int,
          step_init: float = 1.0, grow: float = 1.25, shrink: float = 0.5,
          trace: bool = False, newton_bands: int = 0, newton_steps: int = 0,
          keep: int = 0, min_sep: float = 0.0):
    """Run the ascent for one particle.

    a, b: particle / template coefficients [C] (complex).
    starts: [P, 3] Euler triples.  Returns dict with ``euler`` [P', 3],
    ``score`` [P'], ``best`` (index), and ``trace`` (list of per-band
    [T+1, P'] score arrays) if requested.

    Options beyond the gradient bands described above:
    * newton_bands: the last `newton_bands` bands take Newton steps instead
      (``newton_steps`` of them, or `steps` if 0): each band evaluates
      (S, grad, Hessian) at the carried point, sets mu = 1, then per step
      x' = wrap(x + mu d) with d from ``newton_direction``; accept if
      S(x') >= S(x) (mu <- min(1, mu * grow)), else mu <- mu * shrink.
    * keep > 0 (and < P): after the first band only the restarts chosen by
      ``prune_candidates(keep, min_sep)`` continue (P' = keep).
    """
    x = wrap_many(np.asarray(starts, dtype=np.float64))
    P = x.shape[0]
    S = np.full(P, -np.inf)
    hist = []
    nb = len(bands)
    for bi, L in enumerate(bands):
        xi = sc.cross_power(a, b, idx, L)
        W = sc.curvature_weight(a, b, idx, L)
        eta0 = step_init / W if W > 0 else 0.0
        if bi >= nb - newton_bands:
            T = newton_steps if newton_steps > 0 else steps
            S, G, H = sc.score_grad_hess(xi, x)
            mu = np.ones(P)
            band_hist = [S.copy()]
            for _ in range(T):
                xt = wrap_many(x + mu[:, None] * newton_direction(x, G, H, eta0))
                St, Gt, Ht = sc.score_grad_hess(xi, xt)
                acc = St >= S
                x[acc] = xt[acc]
                S = np.where(acc, St, S)
                G[acc] = Gt[acc]
                H[acc] = Ht[acc]
                mu = np.where(acc, np.minimum(1.0, mu * grow), mu * shrink)
                band_hist.append(S.copy())
        else:
            eta = np.full(P, eta0)
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
        if bi == 0 and 0 < keep < P:
            sel = prune_candidates(x, S, keep, min_sep)
            x, S, P = x[sel], S[sel], keep
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


def align_shifts(vol, b, idx: IndexSet, shifts, bands, starts, steps: int, **kw):
    """Shift search for one particle: for each integer voxel shift d, expand
    the shifted volume f(x + d h) and march from `starts`; the best final
    score wins (first shift on ties).  Returns (euler, score, shift index)."""
    from . import expand
    best = None
    for si, d in enumerate(shifts):
        a = expand.expand(expand.shift_volume(np.asarray(vol, dtype=np.float64), d), idx)
        r = march(a, b, idx, bands, starts, steps, **kw)
        s = r["score"][r["best"]]
        if best is None or s > best[1]:
            best = (r["euler"][r["best"]], s, si)
    return best
