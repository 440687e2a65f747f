"""Krylov evaluation of a linear combination of phi functions -- TEST
INFRASTRUCTURE (plain NumPy / SciPy).

    w = sum_{j=0}^{p} phi_j(h J) b_j h^j

is the first block of exp(h A~) [b_0; e_p] for the augmented matrix
A~ = [[J, B], [0, K]], B = [b_p, ..., b_1], K the p x p shift (the theorem of
Sec. 2.1).  The augmented system w' = A~ w is advanced over [0, h] in
substeps; each substep projects exp(tau A~) onto a Krylov space built by
Arnoldi's process (Sec. 2.1 outline of phipm and KIOPS).  The paper defers
the details to those methods; the readings here:

  * Arnoldi with an orthogonalisation window q: the new vector is
    orthogonalised (classical Gram-Schmidt, one pass) against the last q basis
    vectors only -- KIOPS's incomplete orthogonalisation, q = 2 by default;
    q = 0 means all of them;
  * a fixed Krylov dimension m (default 30); a breakdown (h_{j+1,j} below
    1e-300) ends the basis early, the space then being invariant and the
    projection exact;
  * the substep's result is beta V_m exp(tau H_m) e_1 with the error estimate
    beta h_{m+1,m} tau |e_m^T phi_1(tau H_m) e_1| (Saad's a-posteriori
    estimate), both read off one exponential of the (m+1) x (m+1) matrix
    [[tau H_m, e_1], [0, 0]];
  * a substep is accepted when its estimate is at most tol (tau / h) ||w||
    (its share of the tolerance over the whole interval, relative to the
    current vector); the next step size, after acceptance and after a
    rejection, is 0.9 tau (tol (tau/h) ||w|| / est)^{1/(m+1)}, at most 2 tau
    and at least tau / 10, shortened to end at h; the first tries the whole
    interval; a rejection reuses the basis (the space does not depend on tau);
  * at most max_substeps accepted substeps and 10 * max_substeps attempts.

Only scipy.linalg.expm (Pade scaling and squaring) is used as a library step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg


@dataclass
class KrylovOptions:
    m: int = 30
    window: int = 2
    max_substeps: int = 1000


@dataclass
class KrylovStats:
    substeps: int = 0
    rejections: int = 0
    products: int = 0
    converged: bool = True


def _aug_apply(jv, B, x):
    """A~ x for x = [x_N; y_p]: [J x_N + B y; K y], B = [b_p, ..., b_1]."""
    N = x.shape[0] - len(B)
    p = len(B)
    out = np.empty_like(x)
    xn, y = x[:N], x[N:]
    out[:N] = jv(xn)
    for i in range(p):
        out[:N] += y[i] * B[i]
    if p:
        out[N:N + p - 1] = y[1:]
        out[N + p - 1] = 0.0
    return out


def arnoldi(apply, v, m: int, window: int):
    """Orthonormal basis V (m+1 columns at most) and Hessenberg H of the
    Krylov space of `apply` from v; returns (V, H, m_eff, beta, products)."""
    n = v.shape[0]
    beta = float(np.linalg.norm(v))
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = v / beta
    m_eff = m
    products = 0
    for j in range(m):
        w = apply(V[:, j])
        products += 1
        lo = 0 if window <= 0 else max(0, j - window + 1)
        hs = [float(V[:, i] @ w) for i in range(lo, j + 1)]  # classical Gram-Schmidt, one pass
        for i, hij in zip(range(lo, j + 1), hs):
            H[i, j] = hij
        for i, hij in zip(range(lo, j + 1), hs):
            w = w - hij * V[:, i]
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        if not hn > 1e-300:  # invariant subspace: the projection is exact
            m_eff = j + 1
            break
        V[:, j + 1] = w / hn
    return V, H, m_eff, beta, products


def phi_combination(jv, bs, h: float, tol: float, opt: KrylovOptions | None = None):
    """w = sum_j phi_j(h J) b_j h^j for bs = [b_0, ..., b_p] (None = zero)."""
    opt = opt or KrylovOptions()
    p = len(bs) - 1
    N = next(len(b) for b in bs if b is not None)
    bz = [np.zeros(N) if b is None else np.asarray(b, dtype=np.float64) for b in bs]
    B = [bz[p - i] for i in range(p)]  # [b_p, ..., b_1]
    w = np.zeros(N + p)
    w[:N] = bz[0]
    if p:
        w[N + p - 1] = 1.0
    st = KrylovStats()
    apply = lambda x: _aug_apply(jv, B, x)
    t = 0.0
    tau = h
    attempts = 0
    while t < h:
        if st.substeps >= opt.max_substeps or attempts >= 10 * opt.max_substeps:
            st.converged = False
            break
        beta = float(np.linalg.norm(w))
        if beta == 0.0:
            break
        V, H, m, beta, prods = arnoldi(apply, w, opt.m, opt.window)
        st.products += prods
        exact = m < opt.m  # breakdown: no truncation error
        while True:
            attempts += 1
            tau = min(tau, h - t)
            Mx = np.zeros((m + 1, m + 1))
            Mx[:m, :m] = tau * H[:m, :m]
            Mx[0, m] = 1.0
            E = scipy.linalg.expm(Mx)
            F = E[:m, 0]                       # exp(tau H_m) e_1
            est = 0.0 if exact else beta * H[m, m - 1] * tau * abs(E[m - 1, m])
            allow = tol * (tau / h) * beta
            fac = 2.0 if est == 0.0 else min(2.0, max(0.1, 0.9 * (allow / est) ** (1.0 / (m + 1))))
            if est <= allow:
                w = beta * (V[:, :m] @ F)
                t = h if tau >= h - t else t + tau
                st.substeps += 1
                tau = tau * fac
                break
            st.rejections += 1
            tau = tau * fac
            if attempts >= 10 * opt.max_substeps:
                st.converged = False
                break
        if not st.converged:
            break
    return w[:N], st
