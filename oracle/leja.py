"""Leja interpolation of phi_l(h J) v (Sec. 2.2), its vertical form (Sec. 4) and
substepping on non-convergence (Sec. 2.1 theorem, Sec. 2.2 last paragraph).

Steps, in the paper's order and notation:

1. Spectrum (Sec. 2.2): alpha <= Re sigma(J) <= beta <= 0.  Reading: beta = 0 and
   alpha = -safety * lambda_hat, lambda_hat from power iteration (oracle.power).
2. Scale and shift onto [-2, 2]: c = (alpha + beta)/2 (midpoint), gamma =
   (beta - alpha)/4 (a quarter of the interval length; the printed sentence is
   garbled).
3. Divided differences d_m of phi_l(a tau (c + gamma xi)) at the Leja points xi_m
   (oracle.divdiff), one coefficient set per accumulator.
4. Newton recurrence (Sec. 2.2 display):
        y_0 = v,  p = d_0 v,
        y_m = ((J - c) / gamma - xi_{m-1}) y_{m-1},   p += d_m y_m,
   one J-product per m.  The vertical form (Sec. 4) shares y_m between K
   accumulators that differ only in their coefficients (l_k, a_k).
5. Stop (Sec. 2.2): the error estimate e_m = |d_m| ||y_m||_2 falls below the
   tolerance.  Reading: relative to the current result, e_m <= tol ||p||_2
   (the paper's absolute form e_m <= tol is the relative_tol = False option);
   checked from m = 1 on; each accumulator freezes at its first such m.
6. Reject (Sec. 2.2, last paragraph: large steps need too many points and the
   expansion becomes unreliable).  Reading: an accumulator is rejected when
   m reaches max_points unconverged, when a term exceeds
   hump_max * ||v|| * max_j |f_j| (its data scale, fixed before the loop), or
   when a non-finite value appears.
7. Substepping.  Reading of a conflict: Sec. 2.2 says substepping applies to
   the exponential only, while the spec path asks for it on
   non-convergence.  With w(t) = t^l phi_l(t J) v (the Sec. 2.1 theorem with a
   single b), the exact identity
        w(t + tau) = e^{tau J} w(t) + sum_{j=1..l} tau^j t^{l-j}/(l-j)! phi_j(tau J) v
   lets s substeps of tau = T/s reach w(T) / T^l = phi_l(T J) v.  The
   phi_j(tau J) v, j = 1..l, come from one vertical recurrence; each of the
   s-1 propagations by e^{tau J} is its own recurrence.  Substeps are tried only
   after a rejection: s = 2, 4, ... up to max_substeps.  In a vertical call the
   accumulators that converged are kept and only the rejected ones are redone,
   each on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .divdiff import divided_differences
from .phi import phi
from .points import leja_points
from .power import power_iteration

_XI_CACHE: dict = {}


def xi_table(count: int = 101) -> np.ndarray:
    if count not in _XI_CACHE:
        _XI_CACHE[count] = leja_points(count)
    return _XI_CACHE[count]


@dataclass
class Options:
    """Constants the paper leaves open (readings; see module docstring)."""

    safety: float = 1.25
    power_iters: int = 20
    max_points: int = 100
    hump_max: float = 1e4
    max_substeps: int = 64
    relative_tol: bool = True
    bound: float | None = None      # lambda_hat given: skip power iteration
    substeps: int | None = None     # initial s (a proposal); None = 1
    power_seed: int = 0x5EED


@dataclass
class Recurrence:
    p: list
    converged: list
    m_star: list
    err: list
    reason: list
    iters: int


@dataclass
class Stats:
    m_star: list = field(default_factory=list)
    substeps: list = field(default_factory=list)
    iters_total: int = 0
    power_iters: int = 0
    rejections: int = 0
    bound: float = 0.0
    c: float = 0.0
    gamma: float = 0.0
    err: list = field(default_factory=list)
    converged: bool = True


def interval(lam_hat: float, safety: float):
    """Steps 1-2: (c, gamma) from the bound, alpha = -safety*lambda, beta = 0."""
    alpha = -safety * lam_hat
    beta = 0.0
    c = 0.5 * (alpha + beta)
    gamma = 0.25 * (beta - alpha)
    return c, gamma


def coefficients(l: int, a: float, tau: float, c: float, gamma: float, npts: int):
    """Step 3: d_0..d_{npts-1} of phi_l(a tau (c + gamma xi)) and max_j |f_j|."""
    xi = xi_table(max(npts, 101))[:npts]
    s = a * tau
    f = [phi(l, s * (c + gamma * x)) for x in xi]
    return divided_differences(f, xi), max(abs(x) for x in f)


def newton_recurrence(jv, v, ls, As, tau, c, gamma, tol, opt: Options) -> Recurrence:
    """Steps 4-6 for K accumulators phi_{l_k}(a_k tau J) v sharing y_m."""
    K = len(ls)
    M = opt.max_points
    xi = xi_table(max(M + 1, 101))
    coef = [coefficients(ls[k], As[k], tau, c, gamma, M + 1) for k in range(K)]
    v = np.asarray(v, dtype=np.float64)
    nv = float(np.linalg.norm(v))
    p = [coef[k][0][0] * v for k in range(K)]
    conv = [False] * K
    dead = [False] * K
    m_star = [-1] * K
    err = [math.inf] * K
    reason = ["maxpts"] * K
    if nv == 0.0:
        return Recurrence(p, [True] * K, [0] * K, [0.0] * K, ["ok"] * K, 0)
    y = v.copy()
    iters = 0
    for m in range(1, M + 1):
        y = (jv(y) - c * y) / gamma - xi[m - 1] * y
        iters += 1
        ny = float(np.linalg.norm(y))
        for k in range(K):
            if conv[k] or dead[k]:
                continue
            d_m = coef[k][0][m]
            p[k] = p[k] + d_m * y
            e = abs(d_m) * ny
            npk = float(np.linalg.norm(p[k]))
            if not (math.isfinite(e) and math.isfinite(npk)):
                dead[k], reason[k] = True, "nonfinite"
                continue
            if e > opt.hump_max * nv * coef[k][1]:
                dead[k], reason[k] = True, "hump"
                continue
            bound = tol * npk if opt.relative_tol else tol
            if e <= bound:
                conv[k], m_star[k], err[k], reason[k] = True, m, e, "ok"
        if all(conv[k] or dead[k] for k in range(K)):
            break
    return Recurrence(p, conv, m_star, err, reason, iters)


def _substepped(jv, v, l, T, s_start, c, gamma, tol, opt: Options, st: Stats):
    """Step 7 for one accumulator phi_l(T J) v; returns (w, s, iters, ok)."""
    s = s_start
    w = np.zeros_like(v)
    while s <= opt.max_substeps:
        tau = T / s
        ok = True
        used = 0
        if l == 0:
            w = np.array(v, dtype=np.float64)
            for _ in range(s):
                r = newton_recurrence(jv, w, [0], [1.0], tau, c, gamma, tol, opt)
                used += r.iters
                w = r.p[0]
                if not r.converged[0]:
                    ok = False
                    break
        else:
            r = newton_recurrence(jv, v, list(range(1, l + 1)), [1.0] * l, tau, c, gamma, tol, opt)
            used += r.iters
            P = r.p  # P[j-1] = phi_j(tau J) v
            ok = all(r.converged)
            if ok:
                w = P[l - 1] / float(s) ** l
                for i in range(1, s):
                    r2 = newton_recurrence(jv, w, [0], [1.0], tau, c, gamma, tol, opt)
                    used += r2.iters
                    if not r2.converged[0]:
                        ok = False
                        break
                    w = r2.p[0]
                    for j in range(1, l + 1):
                        w = w + (float(i) ** (l - j) / (math.factorial(l - j) * float(s) ** l)) * P[j - 1]
        st.iters_total += used
        if ok:
            return w, s, used, True
        st.rejections += 1
        s *= 2
    return w, s // 2, 0, False


def phi_vertical(op, v, ls, As, h, tol, opt: Options | None = None):
    """w_k = phi_{l_k}(a_k h J) v, k < K, by Leja interpolation (Sec. 2.2, 4).

    op: object with .jv(x) and .n (oracle.operators.Operator).
    Returns (list of w_k, Stats).
    """
    opt = opt or Options()
    K = len(ls)
    st = Stats(m_star=[-1] * K, substeps=[1] * K, err=[0.0] * K)
    if opt.bound is not None and opt.bound > 0:
        lam = float(opt.bound)
    else:
        lam = power_iteration(op.jv, op.n, opt.power_iters, opt.power_seed)
        st.power_iters = opt.power_iters
    c, gamma = interval(lam, opt.safety)
    st.bound, st.c, st.gamma = lam, c, gamma
    v = np.asarray(v, dtype=np.float64)
    ws = [None] * K
    s0 = opt.substeps if (opt.substeps and opt.substeps > 1) else 1
    pending = list(range(K))
    if s0 == 1:
        r = newton_recurrence(op.jv, v, ls, [float(a) for a in As], h, c, gamma, tol, opt)
        st.iters_total += r.iters
        pending = [k for k in range(K) if not r.converged[k]]
        for k in range(K):
            ws[k] = r.p[k]
            if r.converged[k]:
                st.m_star[k] = r.m_star[k]
                st.err[k] = r.err[k]
        if pending:
            st.rejections += 1
        s0 = 2
    for k in pending:
        w, s, used, ok = _substepped(op.jv, v, ls[k], float(As[k]) * h, s0, c, gamma, tol, opt, st)
        ws[k] = w
        st.substeps[k] = s
        st.m_star[k] = used if ok else -1
        if not ok:
            st.converged = False
    return ws, st


def phi_action(op, v, l, h, tol, opt: Options | None = None):
    """w = phi_l(h J) v (the single-accumulator case of phi_vertical)."""
    ws, st = phi_vertical(op, v, [l], [1.0], h, tol, opt)
    return ws[0], st
