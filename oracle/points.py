"""Leja points on [-2, 2] (Sec. 2.2: the spectrum is mapped onto a pre-computed
Leja sequence in [-2, 2]).

Definition (Leja 1957, as used in Sec. 2.2): xi_0 is a fixed start point and
each further point maximises the product of distances to all earlier points,

    xi_m = argmax_{x in [-2, 2]}  prod_{j<m} |x - xi_j|.

Reading (the paper is silent on the start point and on ties): xi_0 = +2, and
when two maximisers tie the leftmost one is taken (the only exact tie occurs
at m = 3, between +-2/sqrt(3)).

Computation, written for clarity rather than speed: the log of the product,
sum_j log|x - xi_j|, is strictly concave on each gap between consecutive
earlier points (its second derivative is -sum_j 1/(x - xi_j)^2), so each gap
holds exactly one local maximiser, the zero of the derivative
g(x) = sum_j 1/(x - xi_j).  Each zero is found by bisection to full FP64
precision; the end points -2 and +2 are candidates as long as they are not yet
in the sequence.  The global maximiser is the best candidate.
"""
from __future__ import annotations

import math

import numpy as np


def _logprod(x: float, pts: list[float]) -> float:
    s = 0.0
    for p in pts:
        d = abs(x - p)
        if d == 0.0:
            return -math.inf
        s += math.log(d)
    return s


def _gap_roots(lo: np.ndarray, hi: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Zero of g on each open gap (lo_i, hi_i), by bisection, all gaps at once.

    g -> +inf at the left end of a gap and -inf at its right end, so the sign
    of g at the midpoint tells which half holds the zero.  Bisection stops when
    the bracket is two adjacent doubles; the end with the smaller |g| is kept.
    """
    a, b = lo.copy(), hi.copy()
    for _ in range(2000):
        mid = 0.5 * (a + b)
        live = (mid > a) & (mid < b)
        if not live.any():
            break
        g = (1.0 / (mid[:, None] - pts[None, :])).sum(axis=1)
        a = np.where(live & (g >= 0.0), mid, a)
        b = np.where(live & (g <= 0.0), mid, b)
    ga = np.abs((1.0 / (a[:, None] - pts[None, :])).sum(axis=1))
    gb = np.abs((1.0 / (b[:, None] - pts[None, :])).sum(axis=1))
    return np.where(ga <= gb, a, b)


def leja_points(count: int = 101) -> np.ndarray:
    """First `count` Leja points on [-2, 2] with xi_0 = 2 (Sec. 2.2)."""
    pts = [2.0]
    while len(pts) < count:
        srt = sorted(pts)
        cands = []
        if -2.0 not in pts:
            cands.append(-2.0)
        s = np.asarray(srt)
        cands.extend(_gap_roots(s[:-1], s[1:], np.asarray(pts)).tolist())
        vals = [_logprod(x, pts) for x in cands]
        best = max(vals)
        # ties (equal up to rounding of the log-sum) go to the leftmost point
        tie_tol = 1e-12 * max(1.0, abs(best))
        chosen = min(x for x, v in zip(cands, vals) if v >= best - tie_tol)
        pts.append(chosen)
    return np.asarray(pts, dtype=np.float64)
