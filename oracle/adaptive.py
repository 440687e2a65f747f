"""Variable step sizes for the embedded exponential integrators -- TEST
INFRASTRUCTURE (plain NumPy/Python, built on oracle.integrators.step).

Sec. 2.3 (automatic step size control):
  * the traditional controller dt_{n+1} = dt_n (tol / e_n)^{1/(p+1)};
  * the cost controller dt_{n+1} = dt_n * g with s = exp(-alpha tanh(beta D)),
    D = (ln c_n - ln c_{n-1}) / (ln dt_n - ln dt_{n-1}), g = lambda for
    1 <= s < lambda, g = delta for delta <= s < 1, g = s otherwise, with the
    printed constants alpha, beta, lambda, delta;
  * the step size taken is the smaller of the two.

Readings where the text is silent:
  * e_n = ||u_4 - u_3||_2 / ||u_4||_2, the embedded estimate relative to the
    new solution; a step is accepted when e_n <= tol;
  * p is the order of the embedded lower-order solution (3 for EPIRK4s3, its
    LeKry form and EXPRB43), so that e_n ~ dt^{p+1};
  * c_n = the step's cost per unit time: its Jacobian-vector products
    (power iteration + Newton terms of every expansion, substeps included)
    divided by dt_n -- the controller's purpose is the least total cost to
    reach T, and with the raw per-step count it would shrink dt without end
    once the count stops falling with dt;
  * after a rejection the step is retried with 0.9 times the traditional
    controller's size (without the factor, an estimate that falls more slowly
    than dt^{p+1} -- stiff order reduction -- creeps down over many
    rejections); a step whose expansions fail is retried with half the size;
  * the cost controller needs two accepted steps: before that, and when
    dt_n = dt_{n-1} (D undefined), D = 0; e_n = 0 leaves only the cost
    controller (the traditional size is unbounded);
  * the last step is shortened to end exactly at T.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .integrators import step
from .leja import Options
from .operators import Operator

# cost controller constants (Sec. 2.3)
ALPHA = 0.65241444
BETA = 0.26862269
LAMBDA = 1.37412002
DELTA = 0.64446017

EMBEDDED_ORDER = {"EPIRK4S3": 3, "EXPRB43": 3, "EPIRK4S3_LEKRY": 3, "EPIRK4S3A": 3, "EPIRK4S3A_LEKRY": 3}
RETRY_SAFETY = 0.9  # retry after a rejection at 0.9 x the traditional size (a reading; see above)


def traditional_factor(e: float, tol: float, p: int) -> float:
    """(tol / e)^{1/(p+1)}; unbounded for e = 0."""
    if e == 0.0:
        return math.inf
    return (tol / e) ** (1.0 / (p + 1))


def cost_factor(dt: float, dt_prev: float, c: float, c_prev: float) -> float:
    """The cost controller's factor g from two consecutive accepted steps."""
    if dt == dt_prev:
        D = 0.0
    else:
        D = (math.log(c) - math.log(c_prev)) / (math.log(dt) - math.log(dt_prev))
    s = math.exp(-ALPHA * math.tanh(BETA * D))
    if 1.0 <= s < LAMBDA:
        return LAMBDA
    if DELTA <= s < 1.0:
        return DELTA
    return s


@dataclass
class Attempt:
    t: float
    dt: float
    err: float
    cost: int
    accepted: bool


@dataclass
class Run:
    u: np.ndarray
    t: float
    accepted: int = 0
    rejected: int = 0
    products: int = 0
    attempts: list = field(default_factory=list)


def integrate(prob, u0, T: float, dt0: float, tol: float, scheme: str = "EPIRK4S3", leja_tol: float | None = None,
              opt: Options | None = None, max_attempts: int = 10000, make_op=None) -> Run:
    """u(T) of u_t = f(u) from u(0) = u0 with variable steps (Sec. 2.3).
    make_op(u) builds the operator linearised at u (default: the family
    operator of `prob`)."""
    if scheme not in EMBEDDED_ORDER:
        raise ValueError(f"{scheme} has no embedded error estimate")
    p = EMBEDDED_ORDER[scheme]
    lt = leja_tol if leja_tol is not None else tol
    u = np.array(u0, dtype=np.float64)
    run = Run(u=u, t=0.0)
    t, dt = 0.0, float(dt0)
    prev = None  # (dt, cost per unit time) of the last accepted step
    while t < T:
        if len(run.attempts) >= max_attempts:
            raise RuntimeError("too many step attempts")
        last = dt >= T - t
        h = T - t if last else dt
        op = make_op(u) if make_op is not None else Operator(prob, state=u)
        u_new, err, log = step(op, scheme, h, lt, opt)
        ok = all(st.converged for st in log)
        cost = sum(st.iters_total + st.power_iters for st in log)
        run.products += cost
        if not ok:
            run.attempts.append(Attempt(t, h, math.inf, cost, False))
            run.rejected += 1
            dt = 0.5 * h
            continue
        nu = float(np.linalg.norm(u_new))
        e = float(np.linalg.norm(err)) / nu if nu > 0.0 else float(np.linalg.norm(err))
        if e <= tol:
            run.attempts.append(Attempt(t, h, e, cost, True))
            run.accepted += 1
            t = T if last else t + h
            u = u_new
            d_trad = h * traditional_factor(e, tol, p)
            rate = cost / h
            d_cost = h * cost_factor(h, prev[0], rate, prev[1]) if prev is not None else h * cost_factor(h, h, 1, 1)
            prev = (h, rate)
            dt = min(d_trad, d_cost)
        else:
            run.attempts.append(Attempt(t, h, e, cost, False))
            run.rejected += 1
            dt = RETRY_SAFETY * h * traditional_factor(e, tol, p)
    run.u = u
    run.t = t
    return run
