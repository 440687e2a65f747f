"""Exponential-integrator steps built on the Leja action (stage driver).

Sec. 1: u_t = f(u) is linearised at u^n as J(u^n) u + F(u^n) and the
nonlinear remainders enter through R(x) = F(x) - F(u^n).  The schemes:

* EXPRB2: u_out = u + phi_1(h J) h f(u) (the first term of every scheme in
  Sec. 5; exponential Rosenbrock-Euler).
* EXPRB43 (Sec. 5.4 equation): internal stages a (coefficient 1/2) and b, the
  third-order u_3 and the fourth-order u_4 = u_3 + phi_4 term.  phi_1(h/2 J) and
  phi_1(h J) on h f(u) run vertically (Sec. 5.4 text).  'EXPRB43_U3' stops at u_3.
* EPIRK4s3 (Sec. 5.1 equation): phi_1 at 1/8, 1/9 and 1 on h f(u) vertically,
  then phi_3 and phi_4 individually (Sec. 5.1 text).
* EPIRK4S3_LEKRY ("LeKry", Sec. 5.1 text): the same scheme with the two
  internal stages phi_1(h/8 J), phi_1(h/9 J) by Leja (vertical), the third
  stage's phi_1(hJ) h f(u) + phi_3(hJ) D_3 as one augmented exponential by
  Krylov (oracle.krylov), and the phi_4 error term by Leja.
* EPIRK4s3A (Sec. 5.2 equation): the same structure with the internal stages
  at 1/2 and 2/3, u_3 = u + phi_1(hJ) h f + phi_3(hJ) (32 R(a) - 27/2 R(b)) h
  and u_4 = u_3 + phi_4(hJ) (-144 R(a) + 81 R(b)) h; phi_1 at 1/2, 2/3 and 1
  vertically, the rest individually (Sec. 5.2 text).  EPIRK4S3A_LEKRY: its
  LeKry form (Sec. 5.2 text), built like EPIRK4S3_LEKRY.

One spectral bound is computed per step and shared by every action (J is fixed
over the step; Sec. 4: the re-scaling is done once).  err = u_4 - u_3 for the
embedded pairs.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .krylov import KrylovOptions, phi_combination
from .leja import Options, Stats, phi_vertical
from .power import power_iteration


def _bound(op, opt: Options) -> tuple[float, int]:
    if opt.bound is not None and opt.bound > 0:
        return float(opt.bound), 0
    return power_iteration(op.jv, op.n, opt.power_iters, opt.power_seed), opt.power_iters


def step(op, scheme: str, h: float, tol: float, opt: Options | None = None):
    """One step from u = op.state.  Returns (u_out, err or None, list of action stats)."""
    opt = opt or Options()
    u = op.state
    lam, pit = _bound(op, opt)
    o = replace(opt, bound=lam)
    fu = op.rhs(u)
    v = h * fu
    log = []

    def act(vec, ls, As):
        ws, st = phi_vertical(op, vec, ls, As, h, tol, o)
        log.append(st)
        return ws

    if scheme == "EXPRB2":
        (A,) = act(v, [1], [1.0])
        out = (u + A, None)
    elif scheme in ("EXPRB43", "EXPRB43_U3"):
        A, B = act(v, [1, 1], [0.5, 1.0])
        a = u + 0.5 * A
        Ra = op.remainder(a, fu)
        (C,) = act(h * Ra, [1], [1.0])
        b = u + B + C
        Rb = op.remainder(b, fu)
        (D3,) = act(h * (16.0 * Ra - 2.0 * Rb), [3], [1.0])
        u3 = u + B + D3
        if scheme == "EXPRB43_U3":
            out = (u3, None)
        else:
            (D4,) = act(h * (-48.0 * Ra + 12.0 * Rb), [4], [1.0])
            u4 = u3 + D4
            out = (u4, u4 - u3)
    elif scheme == "EPIRK4S3":
        A, B, C = act(v, [1, 1, 1], [1.0 / 8.0, 1.0 / 9.0, 1.0])
        a = u + A / 8.0
        b = u + B / 9.0
        Ra = op.remainder(a, fu)
        Rb = op.remainder(b, fu)
        D3v = h * (1892.0 * Ra + 1458.0 * (Rb - 2.0 * Ra))
        (D3,) = act(D3v, [3], [1.0])
        u3 = u + C + D3
        D4v = h * (-42336.0 * Ra - 34992.0 * (Rb - 2.0 * Ra))
        (D4,) = act(D4v, [4], [1.0])
        u4 = u3 + D4
        out = (u4, u4 - u3)
    elif scheme == "EPIRK4S3_LEKRY":
        A, B = act(v, [1, 1], [1.0 / 8.0, 1.0 / 9.0])
        a = u + A / 8.0
        b = u + B / 9.0
        Ra = op.remainder(a, fu)
        Rb = op.remainder(b, fu)
        D3v = h * (1892.0 * Ra + 1458.0 * (Rb - 2.0 * Ra))
        # phi_1(hJ) (h f) + phi_3(hJ) D3v = sum_j phi_j(hJ) b_j h^j, b_1 = f, b_3 = D3v / h^3
        K3, kst = phi_combination(op.jv, [None, fu, None, D3v / h ** 3], h, tol, KrylovOptions())
        log.append(Stats(m_star=[kst.products], substeps=[kst.substeps], iters_total=kst.products,
                         rejections=kst.rejections, converged=kst.converged))
        u3 = u + K3
        D4v = h * (-42336.0 * Ra - 34992.0 * (Rb - 2.0 * Ra))
        (D4,) = act(D4v, [4], [1.0])
        u4 = u3 + D4
        out = (u4, u4 - u3)
    elif scheme in ("EPIRK4S3A", "EPIRK4S3A_LEKRY"):
        lekry = scheme == "EPIRK4S3A_LEKRY"
        ws = act(v, [1, 1] if lekry else [1, 1, 1], [0.5, 2.0 / 3.0] if lekry else [0.5, 2.0 / 3.0, 1.0])
        A, B = ws[0], ws[1]
        a = u + 0.5 * A
        b = u + (2.0 / 3.0) * B
        Ra = op.remainder(a, fu)
        Rb = op.remainder(b, fu)
        D3v = h * (32.0 * Ra - 13.5 * Rb)
        if lekry:
            K3, kst = phi_combination(op.jv, [None, fu, None, D3v / h ** 3], h, tol, KrylovOptions())
            log.append(Stats(m_star=[kst.products], substeps=[kst.substeps], iters_total=kst.products,
                             rejections=kst.rejections, converged=kst.converged))
            u3 = u + K3
        else:
            (D3,) = act(D3v, [3], [1.0])
            u3 = u + ws[2] + D3
        D4v = h * (-144.0 * Ra + 81.0 * Rb)
        (D4,) = act(D4v, [4], [1.0])
        u4 = u3 + D4
        out = (u4, u4 - u3)
    else:
        raise ValueError(scheme)
    if log:
        log[0].power_iters = pit
    return out[0], out[1], log


def rk_reference(op_factory, u0, T: float, nsteps: int) -> np.ndarray:
    """Classical RK4 with many small steps: a plain reference solution of u_t = f(u)
    used only by order tests (op_factory(u) -> operator linearised at u)."""
    u = np.array(u0, dtype=np.float64)
    dt = T / nsteps
    f = lambda w: op_factory(w).rhs(w)  # noqa: E731
    for _ in range(nsteps):
        k1 = f(u)
        k2 = f(u + 0.5 * dt * k1)
        k3 = f(u + 0.5 * dt * k2)
        k4 = f(u + dt * k3)
        u = u + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return u
