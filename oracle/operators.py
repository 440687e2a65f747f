"""Right-hand sides f(u) and Jacobian actions J(u)v of the test problems.

Sec. 3: every spatial derivative is discretised with second-order centred
differences.  The problems run on periodic grids, except the advection-
diffusion-reaction equation, which keeps the paper's homogeneous Neumann
boundaries: on its cell-centred grid the ghost value beyond a boundary face
equals the cell inside it (a reading: the paper does not state its grid or
boundary discretisation), so the boundary rows of the second difference read
(u_1 - u_0)/dx^2 and those of the first difference (u_1 - u_0)/(2 dx).  Sec. 1 writes the
linearisation u_t = J(u^n) u + F(u^n); Sec. 2 and 4 apply J matrix-free.

Reading of the Jacobian action: the paper computes J v "numerically" from RHS
evaluations (Sec. 4); the oracle uses the exact (analytic) Jacobian of the
semi-discrete right-hand side, applied as a stencil, because a finite-
difference directional derivative carries an O(1e-8) error that would swamp a
1e-10 comparison.

Layout: grids are row-major (x fastest); a two-component state is interleaved
(u, v) per grid point.  Each stencil is written with np.roll on a 2D view:
roll(V, +1, axis=1)[j, i] = V[j, i-1] (west), roll(V, -1, axis=1) = east,
roll(V, +1, axis=0) = south, roll(V, -1, axis=0) = north.
"""
from __future__ import annotations

import numpy as np


def _grid(v, nx, ny):
    return np.asarray(v, dtype=np.float64).reshape(ny, nx)


def laplacian(v, nx, ny, dx, dy) -> np.ndarray:
    """Periodic 5-point Laplacian (Sec. 3: centred second differences)."""
    V = _grid(v, nx, ny)
    lx = (np.roll(V, 1, axis=1) - 2.0 * V + np.roll(V, -1, axis=1)) / (dx * dx)
    ly = (np.roll(V, 1, axis=0) - 2.0 * V + np.roll(V, -1, axis=0)) / (dy * dy)
    return (lx + ly).ravel()


def ddx(v, nx, ny, dx) -> np.ndarray:
    """Periodic centred first difference in x: (v_{i+1} - v_{i-1}) / (2 dx)."""
    V = _grid(v, nx, ny)
    return ((np.roll(V, -1, axis=1) - np.roll(V, 1, axis=1)) / (2.0 * dx)).ravel()


def ddy(v, nx, ny, dy) -> np.ndarray:
    V = _grid(v, nx, ny)
    return ((np.roll(V, -1, axis=0) - np.roll(V, 1, axis=0)) / (2.0 * dy)).ravel()


def _neumann_neighbours(v, nx, ny):
    """West, east, south and north values of every point with the boundary
    cells' ghosts equal to the cells themselves (edge replication)."""
    P = np.pad(_grid(v, nx, ny), 1, mode="edge")
    return P[1:-1, :-2], P[1:-1, 2:], P[:-2, 1:-1], P[2:, 1:-1]


def laplacian_neumann(v, nx, ny, dx, dy) -> np.ndarray:
    """5-point Laplacian with homogeneous Neumann boundaries (cell-centred)."""
    V = _grid(v, nx, ny)
    w, e, s, n = _neumann_neighbours(v, nx, ny)
    return ((w - 2.0 * V + e) / (dx * dx) + (s - 2.0 * V + n) / (dy * dy)).ravel()


def grad_sum_neumann(v, nx, ny, dx, dy) -> np.ndarray:
    """d_x v + d_y v by centred differences with homogeneous Neumann boundaries."""
    w, e, s, n = _neumann_neighbours(v, nx, ny)
    return ((e - w) / (2.0 * dx) + (n - s) / (2.0 * dy)).ravel()


class Operator:
    """f(u) and J(state) v of one problem (workloads.Problem)."""

    def __init__(self, prob, state=None):
        self.p = prob
        self.kind = prob.kind
        self.state = prob.state if state is None else np.asarray(state, dtype=np.float64)

    @property
    def n(self):
        return self.p.n

    # --- right-hand side f(u) -------------------------------------------
    def rhs(self, u) -> np.ndarray:
        p = self.p
        u = np.asarray(u, dtype=np.float64)
        nx, ny, dx, dy = p.nx, p.ny, p.dx, p.dy
        if self.kind == "diag":
            return self.state * u
        if self.kind == "advdiff":
            nu, ax, ay = p.coef
            return nu * laplacian(u, nx, ny, dx, dy) - ax * ddx(u, nx, ny, dx) - ay * ddy(u, nx, ny, dy)
        if self.kind == "allencahn":
            (eps,) = p.coef
            return eps * laplacian(u, nx, ny, dx, dy) + u - u ** 3
        if self.kind == "brusselator":
            Du, Dv, a, b = p.coef
            U = u[0::2]
            V = u[1::2]
            out = np.empty_like(u)
            out[0::2] = Du * laplacian(U, nx, ny, dx, dy) + a - (b + 1.0) * U + U * U * V
            out[1::2] = Dv * laplacian(V, nx, ny, dx, dy) + b * U - U * U * V
            return out
        if self.kind == "burgers":
            (nu,) = p.coef
            q = u * u
            return nu * laplacian(u, nx, ny, dx, dy) - 0.5 * (ddx(q, nx, ny, dx) + ddy(q, nx, ny, dy))
        if self.kind == "grayscott":
            # Sec. 3: u_t = a1 Lap u - u v^2 + a (1 - u), v_t = a2 Lap v + u v^2 - (a + b) v
            a1, a2, a, b = p.coef
            U = u[0::2]
            V = u[1::2]
            out = np.empty_like(u)
            out[0::2] = a1 * laplacian(U, nx, ny, dx, dy) - U * V * V + a * (1.0 - U)
            out[1::2] = a2 * laplacian(V, nx, ny, dx, dy) + U * V * V - (a + b) * V
            return out
        if self.kind == "adr":
            # Sec. 3: u_t = alpha Lap u + beta grad u + rate u (1 - u)(u - 1/2); the
            # advection term read as beta (d_x u + d_y u)
            alpha, beta, rate = p.coef
            return (alpha * laplacian_neumann(u, nx, ny, dx, dy) + beta * grad_sum_neumann(u, nx, ny, dx, dy)
                    + rate * u * (1.0 - u) * (u - 0.5))
        raise ValueError(self.kind)

    # --- Jacobian action J(state) v --------------------------------------
    def jv(self, v) -> np.ndarray:
        p = self.p
        v = np.asarray(v, dtype=np.float64)
        nx, ny, dx, dy = p.nx, p.ny, p.dx, p.dy
        s = self.state
        if self.kind == "diag":
            return s * v
        if self.kind == "advdiff":
            nu, ax, ay = p.coef
            return nu * laplacian(v, nx, ny, dx, dy) - ax * ddx(v, nx, ny, dx) - ay * ddy(v, nx, ny, dy)
        if self.kind == "allencahn":
            (eps,) = p.coef
            return eps * laplacian(v, nx, ny, dx, dy) + (1.0 - 3.0 * s * s) * v
        if self.kind == "brusselator":
            Du, Dv, a, b = p.coef
            U, V = s[0::2], s[1::2]
            du, dv = v[0::2], v[1::2]
            out = np.empty_like(v)
            # d/du of (a - (b+1)u + u^2 v) = -(b+1) + 2uv ; d/dv = u^2
            out[0::2] = Du * laplacian(du, nx, ny, dx, dy) + (-(b + 1.0) + 2.0 * U * V) * du + U * U * dv
            # d/du of (b u - u^2 v) = b - 2uv ; d/dv = -u^2
            out[1::2] = Dv * laplacian(dv, nx, ny, dx, dy) + (b - 2.0 * U * V) * du - U * U * dv
            return out
        if self.kind == "burgers":
            (nu,) = p.coef
            q = s * v  # d/du of u^2/2 applied to v
            return nu * laplacian(v, nx, ny, dx, dy) - (ddx(q, nx, ny, dx) + ddy(q, nx, ny, dy))
        if self.kind == "grayscott":
            a1, a2, a, b = p.coef
            U, V = s[0::2], s[1::2]
            du, dv = v[0::2], v[1::2]
            out = np.empty_like(v)
            # d/du of (-u v^2 + a(1 - u)) = -v^2 - a ; d/dv = -2uv
            out[0::2] = a1 * laplacian(du, nx, ny, dx, dy) + (-(V * V) - a) * du - 2.0 * U * V * dv
            # d/du of (u v^2 - (a + b) v) = v^2 ; d/dv = 2uv - (a + b)
            out[1::2] = a2 * laplacian(dv, nx, ny, dx, dy) + V * V * du + (2.0 * U * V - (a + b)) * dv
            return out
        if self.kind == "adr":
            alpha, beta, rate = p.coef
            # d/du of u (1 - u)(u - 1/2) = -3u^2 + 3u - 1/2
            return (alpha * laplacian_neumann(v, nx, ny, dx, dy) + beta * grad_sum_neumann(v, nx, ny, dx, dy)
                    + rate * (-3.0 * s * s + 3.0 * s - 0.5) * v)
        raise ValueError(self.kind)

    def remainder(self, x, fu=None) -> np.ndarray:
        """R(x) = F(x) - F(u) with F(w) = f(w) - J(u) w (Sec. 1), i.e.
        R(x) = f(x) - f(u) - J(u)(x - u), u being the linearisation state."""
        if fu is None:
            fu = self.rhs(self.state)
        return self.rhs(x) - fu - self.jv(np.asarray(x) - self.state)

    def dense(self) -> np.ndarray:
        """J assembled column by column from J e_i (small grids only)."""
        n = self.n
        A = np.empty((n, n))
        e = np.zeros(n)
        for i in range(n):
            e[i] = 1.0
            A[:, i] = self.jv(e)
            e[i] = 0.0
        return A
