"""The 1-D semilinear parabolic problem of Sec. 3 -- TEST INFRASTRUCTURE
(plain NumPy).

    u_t = u_xx + int_0^1 u dx + Phi(x, t),  x in [0, 1],  u(0, t) = u(1, t) = 0,

with Phi chosen so that u = x (1 - x) e^t is the exact solution:
Phi = u_t - u_xx - int u = e^t (x (1 - x) + 2 - 1/6).

Readings (the paper gives the equation, the boundary conditions and the exact
solution only):
  * grid x_i = i dx, i = 1..N, dx = 1/(N + 1), N odd;
  * u_xx by the centred second difference with the boundary values 0;
  * int_0^1 u dx by the composite Simpson rule on the N + 1 intervals (the
    boundary values are 0).  Both are exact for quadratics, so the sampled
    exact solution solves the semi-discrete system exactly and the error left
    after integrating to t is the time integrator's alone -- an end-to-end
    check of the schemes against the paper's closed form;
  * the forcing depends on t, the schemes of Sec. 5 are written for
    autonomous systems: t is carried as an extra unknown tau with tau' = 1
    (state (u_1..u_N, tau), n = N + 1).  The Jacobian at (u, tau) maps
    (v, v_tau) to (v_xx + int v dx + dPhi/dt v_tau, 0), dPhi/dt = Phi.
"""
from __future__ import annotations

import numpy as np


class Semilinear:
    """f, J and R of the augmented semi-discrete system (linearised at `state`)."""

    def __init__(self, N: int, state=None):
        if N < 1 or N % 2 == 0:
            raise ValueError("N must be odd (Simpson's rule on N + 1 intervals)")
        self.N = N
        self.n = N + 1
        self.dx = 1.0 / (N + 1)
        self.x = np.arange(1, N + 1) * self.dx
        # Simpson weights of the interior points (dx/3) (4, 2, 4, ..., 2, 4)
        self.w = np.where(np.arange(1, N + 1) % 2 == 1, 4.0, 2.0) * self.dx / 3.0
        self.g = self.x * (1.0 - self.x) + 11.0 / 6.0  # Phi(x, t) = e^t g(x)
        self.state = None if state is None else np.asarray(state, dtype=np.float64)

    def second_difference(self, u) -> np.ndarray:
        p = np.concatenate(([0.0], u, [0.0]))
        return (p[:-2] - 2.0 * p[1:-1] + p[2:]) / (self.dx * self.dx)

    def rhs(self, U) -> np.ndarray:
        U = np.asarray(U, dtype=np.float64)
        u, t = U[:-1], U[-1]
        out = np.empty_like(U)
        out[:-1] = self.second_difference(u) + self.w @ u + np.exp(t) * self.g
        out[-1] = 1.0
        return out

    def jv(self, V) -> np.ndarray:
        V = np.asarray(V, dtype=np.float64)
        v, vt = V[:-1], V[-1]
        out = np.empty_like(V)
        out[:-1] = self.second_difference(v) + self.w @ v + np.exp(self.state[-1]) * self.g * vt
        out[-1] = 0.0
        return out

    def remainder(self, X, fu=None) -> np.ndarray:
        """R(x) = f(x) - f(u) - J(u)(x - u) (Sec. 1)."""
        if fu is None:
            fu = self.rhs(self.state)
        return self.rhs(X) - fu - self.jv(np.asarray(X) - self.state)

    def exact(self, t: float) -> np.ndarray:
        """The paper's exact solution sampled on the grid, with tau = t."""
        return np.concatenate((self.x * (1.0 - self.x) * np.exp(t), [t]))


def integrate_fixed(N: int, scheme: str, T: float, nsteps: int, tol: float, step_fn, bound_fn):
    """nsteps steps of size T/nsteps from the exact initial state; returns the
    final state.  step_fn(op, scheme, h, tol, bound) -> (U, err, log), bound_fn(op)."""
    U = Semilinear(N).exact(0.0)
    h = T / nsteps
    logs = []
    for _ in range(nsteps):
        op = Semilinear(N, U)
        U, _, log = step_fn(op, scheme, h, tol, bound_fn(op))
        logs.append(log)
    return U, logs
