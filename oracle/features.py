"""Features of the learned proposal -- TEST INFRASTRUCTURE (plain FP64 NumPy).

The learned form (not in the paper; it replaces the power iteration of
Sec. 2.2 and the rejected expansions of its last paragraph when it can)
predicts the spectral bound and the substep count of a phi_l(hJ)v action from
16 dimensionless numbers of the operator, the state and h.  This module is the
plain definition the HIP feature kernel is checked against.

Scales of one problem (grid spacing dx, dy; diffusion coefficient D):
  sigma = D (1/dx^2 + 1/dy^2)           diffusive rate
  A                                    advective rate: |a_x|/dx + |a_y|/dy for
                                       advection-diffusion, |beta| (1/dx + 1/dy)
                                       for advection-diffusion-reaction,
                                       max|u| (1/dx + 1/dy) for Burgers, 0
                                       otherwise
  r(x)                                 local reaction rate of J: 1 - 3u^2
                                       (Allen-Cahn), -(d_x u + d_y u) with centred
                                       differences (Burgers), -(b+1) + 2uv
                                       (Brusselator, first species), -v^2 - a
                                       (Gray-Scott, first species),
                                       rate (-3u^2 + 3u - 1/2) (adv.-diff.-
                                       reaction), 0 otherwise
  D = nu (adv.-diff., Burgers), eps (Allen-Cahn), max(Du, Dv) (Brusselator),
  max(a1, a2) (Gray-Scott), alpha (adv.-diff.-reaction);
  for a diagonal operator sigma = max|lambda| and A = r = 0.
  G                                    Gershgorin bound of the spectral radius
                                       of J: the largest over rows i of
                                       sum_j |J_ij|, J the Jacobian of the
                                       operator's 5-point discretisation at
                                       the state (entries of one row that
                                       fall on the same grid point -- a
                                       Neumann boundary cell's own neighbour
                                       -- summed before the absolute value).
State statistics (first component u, over all grid points): mean, standard
deviation (population), max|u|, and g = max |grad u| dx in grid units,
g = max sqrt(((u_E - u_W)/2)^2 + ((u_N - u_S)/2)^2), neighbours taken as the
operator takes them (periodic, or the boundary cell itself for Neumann).

features[0..15] =
  log10(h G), l/4, log10(1 + A/sigma), log10(1 + max(r_max,0)/sigma),
  log10(1 + max(-r_min,0)/sigma), log10(1 + h A), log10(1 + h max(r_max,0)),
  log10(1 + h max(-r_min,0)), mean/max|u|, std/max|u|, log10(1 + max|u|),
  log10(1 + g), log10(nx ny)/7, log10(dx/dy), log10(G/sigma), ncomp - 1
(the state ratios are 0 for an operator without state or a zero state).

Targets of the network: ln(bound / G) (a correction of the Gershgorin bound)
and log2(accepted substeps).
"""
from __future__ import annotations

import math

import numpy as np

NFEAT = 16


def scales(prob):
    """(sigma, A, r) of a workloads.Problem; r is an array over grid points (or None)."""
    kind, nx, ny = prob.kind, prob.nx, prob.ny
    if kind == "diag":
        lam = np.asarray(prob.state, dtype=np.float64)
        return float(np.max(np.abs(lam))), 0.0, None
    dx, dy = prob.dx, prob.dy
    c = prob.coef
    if kind == "advdiff":
        D = c[0]
        A = abs(c[1]) / dx + abs(c[2]) / dy
        r = None
    elif kind == "allencahn":
        D = c[0]
        u = np.asarray(prob.state, dtype=np.float64)
        A = 0.0
        r = 1.0 - 3.0 * u * u
    elif kind == "burgers":
        D = c[0]
        U = np.asarray(prob.state, dtype=np.float64).reshape(ny, nx)
        A = float(np.max(np.abs(U))) * (1.0 / dx + 1.0 / dy)
        dudx = (np.roll(U, -1, axis=1) - np.roll(U, 1, axis=1)) / (2.0 * dx)
        dudy = (np.roll(U, -1, axis=0) - np.roll(U, 1, axis=0)) / (2.0 * dy)
        r = -(dudx + dudy).ravel()
    elif kind == "brusselator":
        D = max(c[0], c[1])
        st = np.asarray(prob.state, dtype=np.float64)
        u, v = st[0::2], st[1::2]
        A = 0.0
        r = -(c[3] + 1.0) + 2.0 * u * v
    elif kind == "grayscott":
        D = max(c[0], c[1])
        st = np.asarray(prob.state, dtype=np.float64)
        v = st[1::2]
        A = 0.0
        r = -(v * v) - c[2]
    elif kind == "adr":
        D = c[0]
        u = np.asarray(prob.state, dtype=np.float64)
        A = abs(c[1]) * (1.0 / dx + 1.0 / dy)
        r = c[2] * (-3.0 * u * u + 3.0 * u - 0.5)
    else:
        raise ValueError(kind)
    sigma = D * (1.0 / (dx * dx) + 1.0 / (dy * dy))
    return sigma, A, r


def _row_sums(places, cols, extra=()):
    """sum over the distinct columns of a row of |sum of its entries there|:
    places = list of coefficient arrays (one per stencil place), cols = the
    grid point each place falls on; extra = coefficients on columns of their
    own (the other component at the same point)."""
    total = np.zeros_like(places[0])
    for t in range(len(places)):
        first = np.ones(places[0].shape, dtype=bool)
        for t2 in range(t):
            first &= cols[t2] != cols[t]
        same = np.zeros_like(places[0])
        for t2 in range(len(places)):
            same = same + np.where(cols[t2] == cols[t], places[t2], 0.0)
        total = total + np.where(first, np.abs(same), 0.0)
    for e in extra:
        total = total + np.abs(e)
    return total


def gershgorin(prob) -> float:
    """G: the largest absolute row sum of J at the problem's state."""
    kind, nx, ny = prob.kind, prob.nx, prob.ny
    if kind == "diag":
        return float(np.max(np.abs(np.asarray(prob.state, dtype=np.float64))))
    dx, dy = prob.dx, prob.dy
    c = prob.coef
    ix2, iy2 = 1.0 / (dx * dx), 1.0 / (dy * dy)
    i2x, i2y = 1.0 / (2.0 * dx), 1.0 / (2.0 * dy)
    j, i = np.divmod(np.arange(nx * ny), nx)
    if kind == "adr":  # homogeneous Neumann: the ghost beyond a boundary face is the cell itself
        cw = j * nx + np.maximum(i - 1, 0)
        ce = j * nx + np.minimum(i + 1, nx - 1)
        cs = np.maximum(j - 1, 0) * nx + i
        cn = np.minimum(j + 1, ny - 1) * nx + i
    else:
        cw = j * nx + (i - 1) % nx
        ce = j * nx + (i + 1) % nx
        cs = ((j - 1) % ny) * nx + i
        cn = ((j + 1) % ny) * nx + i
    cols = [np.arange(nx * ny), cw, ce, cs, cn]
    one = np.ones(nx * ny)

    def lap(D):  # D times the 5-point Laplacian: centre, W, E, S, N
        return [-2.0 * D * (ix2 + iy2) * one, D * ix2 * one, D * ix2 * one, D * iy2 * one, D * iy2 * one]

    if kind == "advdiff":
        nu, ax, ay = c[0], c[1], c[2]
        pl = lap(nu)
        pl[1] = pl[1] + ax * i2x
        pl[2] = pl[2] - ax * i2x
        pl[3] = pl[3] + ay * i2y
        pl[4] = pl[4] - ay * i2y
        return float(np.max(_row_sums(pl, cols)))
    if kind == "allencahn":
        u = np.asarray(prob.state, dtype=np.float64)
        pl = lap(c[0])
        pl[0] = pl[0] + 1.0 - 3.0 * u * u
        return float(np.max(_row_sums(pl, cols)))
    if kind == "burgers":  # nu Lap x - (d/dx + d/dy)(u x), centred differences
        u = np.asarray(prob.state, dtype=np.float64)
        pl = lap(c[0])
        pl[1] = pl[1] + u[cw] * i2x
        pl[2] = pl[2] - u[ce] * i2x
        pl[3] = pl[3] + u[cs] * i2y
        pl[4] = pl[4] - u[cn] * i2y
        return float(np.max(_row_sums(pl, cols)))
    if kind == "adr":  # alpha Lap x + beta (d/dx + d/dy) x + rate (3u - 3u^2 - 1/2) x
        u = np.asarray(prob.state, dtype=np.float64)
        al, be, rate = c[0], c[1], c[2]
        pl = lap(al)
        pl[0] = pl[0] + rate * (3.0 * u - 3.0 * u * u - 0.5)
        pl[1] = pl[1] - be * i2x
        pl[2] = pl[2] + be * i2x
        pl[3] = pl[3] - be * i2y
        pl[4] = pl[4] + be * i2y
        return float(np.max(_row_sums(pl, cols)))
    st = np.asarray(prob.state, dtype=np.float64)
    U, V = st[0::2], st[1::2]
    if kind == "brusselator":  # f = a - (b+1)u + u^2 v, g = b u - u^2 v
        Du, Dv, b = c[0], c[1], c[3]
        pu = lap(Du)
        pu[0] = pu[0] - (b + 1.0) + 2.0 * U * V
        pv = lap(Dv)
        pv[0] = pv[0] - U * U
        ru = _row_sums(pu, cols, extra=(U * U,))
        rv = _row_sums(pv, cols, extra=(b - 2.0 * U * V,))
        return float(max(np.max(ru), np.max(rv)))
    if kind == "grayscott":  # f = -u v^2 + a(1 - u), g = u v^2 - (a + b) v
        a1, a2, a, b = c[0], c[1], c[2], c[3]
        pu = lap(a1)
        pu[0] = pu[0] - V * V - a
        pv = lap(a2)
        pv[0] = pv[0] + 2.0 * U * V - (a + b)
        ru = _row_sums(pu, cols, extra=(-2.0 * U * V,))
        rv = _row_sums(pv, cols, extra=(V * V,))
        return float(max(np.max(ru), np.max(rv)))
    raise ValueError(kind)


def state_stats(prob):
    """(mean, std, max|u|, g) of the first state component; zeros without state."""
    if prob.kind in ("advdiff", "diag") or prob.state is None:
        return 0.0, 0.0, 0.0, 0.0
    st = np.asarray(prob.state, dtype=np.float64)
    u = st[0::prob.ncomp]
    U = u.reshape(prob.ny, prob.nx)
    if prob.kind == "adr":  # Neumann: a boundary cell is its own ghost neighbour
        P = np.pad(U, 1, mode="edge")
        gx = (P[1:-1, 2:] - P[1:-1, :-2]) / 2.0
        gy = (P[2:, 1:-1] - P[:-2, 1:-1]) / 2.0
    else:
        gx = (np.roll(U, -1, axis=1) - np.roll(U, 1, axis=1)) / 2.0
        gy = (np.roll(U, -1, axis=0) - np.roll(U, 1, axis=0)) / 2.0
    g = float(np.max(np.sqrt(gx * gx + gy * gy)))
    return float(np.mean(u)), float(np.std(u)), float(np.max(np.abs(u))), g


def features(prob, h: float, l: int) -> np.ndarray:
    """The 16 features of (operator at state, h, l), in FP64."""
    sigma, A, r = scales(prob)
    G = gershgorin(prob)
    rmax = float(np.max(r)) if r is not None else 0.0
    rmin = float(np.min(r)) if r is not None else 0.0
    mean, std, umax, g = state_stats(prob)
    dx = prob.dx if prob.kind != "diag" else 1.0
    dy = prob.dy if prob.kind != "diag" else 1.0
    den = umax if umax > 0.0 else math.inf
    f = [
        math.log10(h * G),
        l / 4.0,
        math.log10(1.0 + A / sigma),
        math.log10(1.0 + max(rmax, 0.0) / sigma),
        math.log10(1.0 + max(-rmin, 0.0) / sigma),
        math.log10(1.0 + h * A),
        math.log10(1.0 + h * max(rmax, 0.0)),
        math.log10(1.0 + h * max(-rmin, 0.0)),
        mean / den,
        std / den,
        math.log10(1.0 + umax),
        math.log10(1.0 + g),
        math.log10(prob.nx * prob.ny) / 7.0,
        math.log10(dx / dy),
        math.log10(G / sigma),
        float(prob.ncomp - 1),
    ]
    return np.asarray(f, dtype=np.float64)


def targets(prob, bound: float, substeps: int) -> np.ndarray:
    """(ln(bound / G), log2(substeps))."""
    return np.asarray([math.log(bound / gershgorin(prob)), math.log2(substeps)], dtype=np.float64)
