"""Seeded problem instances for the Leja phi-action workloads.

Every instance is a 2D grid problem of one of the families the paper uses as
test problems (Section 3: advection-diffusion, Allen-Cahn, Brusselator,
Gray-Scott, and the advection-diffusion-reaction equation, the last with
homogeneous Neumann boundaries on a cell-centred grid, the others periodic;
Burgers and a diagonal operator are added as a further family and as a
closed-form check).  Grids are row-major with x fastest; two-component states are
interleaved (u, v) per grid point.

Only random draws and parameter bookkeeping live here: the operators, the
right-hand sides and the method itself are implemented separately by the
oracle and by the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KINDS = ("diag", "advdiff", "allencahn", "brusselator", "burgers", "grayscott", "adr")


@dataclass
class Problem:
    """A linearisation point of one PDE family on a 2D grid (periodic; 'adr':
    homogeneous Neumann boundaries, cell-centred).

    kind   : one of KINDS
    nx, ny : grid points per axis
    ncomp  : components per grid point (2 for the Brusselator, else 1)
    dx, dy : grid spacing
    coef   : family parameters (see the constructors below for the order)
    state  : the state u at which the Jacobian is taken (flat float64,
             length nx*ny*ncomp); for 'diag' the diagonal itself; None for the
             linear advection-diffusion operator
    h_cfl  : the explicit (forward-Euler) diffusive stability step dx^2/(4 D)
    """

    kind: str
    nx: int
    ny: int
    ncomp: int
    dx: float
    dy: float
    coef: tuple
    state: np.ndarray | None
    h_cfl: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.ncomp


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_vector(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """n float64 draws from U[lo, hi) with PCG64(seed)."""
    return _rng(seed).uniform(lo, hi, size=n).astype(np.float64)


def diag_problem(n: int, lam_min: float, seed: int) -> Problem:
    """Diagonal operator J = diag(lambda), lambda ~ U[lam_min, 0] (lam_min < 0)."""
    lam = _rng(seed).uniform(lam_min, 0.0, size=n)
    return Problem("diag", n, 1, 1, 1.0, 1.0, (), lam.astype(np.float64), 1.0 / abs(lam_min))


def advdiff_bump(n: int = 32, nu: float = 1.0, peclet: float = 1.0, seed: int = 1,
                 sigma: float = 0.1, noise: float = 1e-3):
    """Linear advection-diffusion u_t = nu*Lap(u) - a.grad(u) on [0,1)^2.

    The velocity a_x = a_y = peclet*nu/dx gives grid Peclet number |a| dx / nu
    = peclet per axis.  Returns (problem, v) where v is a Gaussian bump of
    width sigma at a random centre (periodic minimum-image distance) plus
    U[0, noise) noise.  coef = (nu, a_x, a_y).
    """
    dx = 1.0 / n
    a = peclet * nu / dx
    rng = _rng(seed)
    cx, cy = rng.uniform(0.0, 1.0, size=2)
    x = (np.arange(n) + 0.0) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")  # X[j, i] = x_i, row j = y_j
    ddx = np.abs(X - cx)
    ddx = np.minimum(ddx, 1.0 - ddx)
    ddy = np.abs(Y - cy)
    ddy = np.minimum(ddy, 1.0 - ddy)
    v = np.exp(-(ddx ** 2 + ddy ** 2) / (2.0 * sigma ** 2))
    v = v + rng.uniform(0.0, noise, size=v.shape)
    prob = Problem("advdiff", n, n, 1, dx, dx, (nu, a, a), None, dx * dx / (4.0 * nu),
                   meta={"centre": (cx, cy)})
    return prob, v.ravel().astype(np.float64)


def allen_cahn_noise(n: int = 512, eps: float = 1e-3, seed: int = 2, amp: float = 0.1) -> Problem:
    """Allen-Cahn u_t = eps*Lap(u) + u - u^3 on [-1,1)^2 (Section 3), periodic.

    u0 ~ U[-amp, amp].  coef = (eps,).
    """
    dx = 2.0 / n
    u = _rng(seed).uniform(-amp, amp, size=n * n)
    return Problem("allencahn", n, n, 1, dx, dx, (eps,), u.astype(np.float64), dx * dx / (4.0 * eps))


def brusselator_perturbed(n: int = 1024, D: float = 2e-3, a: float = 1.0, b: float = 3.0,
                          seed: int = 3, amp: float = 1e-2) -> Problem:
    """Brusselator u_t = D Lap u + a - (b+1)u + u^2 v, v_t = D Lap v + b u - u^2 v on [0,1)^2.

    State interleaved (u, v) per point, perturbed by amp*U[-1,1] about the
    steady state (a, b/a).  coef = (D_u, D_v, a, b).
    """
    dx = 1.0 / n
    rng = _rng(seed)
    st = np.empty((n * n, 2))
    st[:, 0] = a + amp * rng.uniform(-1.0, 1.0, size=n * n)
    st[:, 1] = b / a + amp * rng.uniform(-1.0, 1.0, size=n * n)
    return Problem("brusselator", n, n, 2, dx, dx, (D, D, a, b), st.ravel(), dx * dx / (4.0 * D))


def gray_scott_spots(n: int = 1024, a1: float = 1e-3, a2: float = 1e-3, a: float = 0.04, b: float = 0.06,
                     seed: int = 8, amp: float = 0.0) -> Problem:
    """Gray-Scott u_t = a1 Lap u - u v^2 + a(1 - u), v_t = a2 Lap v + u v^2 - (a + b) v
    on [0,1)^2, periodic (Sec. 3), with the initial state of Sec. 3:
    u = 1 - exp(-150((x-1/2)^2 + (y-1/2)^2)), v = exp(-150((x-1/2)^2 + 2(y-1/2)^2)),
    plus amp U[-1,1] noise (seeded).  State interleaved (u, v).  coef = (a1, a2, a, b)."""
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)  # row = y, column = x
    u = 1.0 - np.exp(-150.0 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))
    v = np.exp(-150.0 * ((X - 0.5) ** 2 + 2.0 * (Y - 0.5) ** 2))
    st = np.empty((n * n, 2))
    st[:, 0] = u.ravel()
    st[:, 1] = v.ravel()
    if amp > 0.0:
        st += amp * _rng(seed).uniform(-1.0, 1.0, size=st.shape)
    D = max(a1, a2)
    return Problem("grayscott", n, n, 2, dx, dx, (a1, a2, a, b), st.ravel(), dx * dx / (4.0 * D))


def adr_neumann(n: int = 256, alpha: float = 1e-2, beta: float = -10.0, rate: float = 100.0,
                seed: int = 9, amp: float = 0.0) -> Problem:
    """Advection-diffusion-reaction u_t = alpha Lap u + beta (d_x + d_y) u + rate u (1 - u)(u - 1/2)
    on [0,1]^2 with homogeneous Neumann boundaries (Sec. 3), on the cell-centred
    grid x_i = (i + 1/2)/n, with the initial state of Sec. 3,
    u = 256 (x y (1 - x)(1 - y))^2 + 0.3, plus amp U[-1,1] noise (seeded).
    coef = (alpha, beta, rate)."""
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(x, x)  # row = y, column = x
    u = 256.0 * (X * Y * (1.0 - X) * (1.0 - Y)) ** 2 + 0.3
    if amp > 0.0:
        u = u + amp * _rng(seed).uniform(-1.0, 1.0, size=u.shape)
    return Problem("adr", n, n, 1, dx, dx, (alpha, beta, rate), u.ravel().astype(np.float64),
                   dx * dx / (4.0 * alpha))


def fourier_modes(n: int, count: int = 3, seed: int = 11, kmax: int = 40):
    """v[j, i] = sum_k A_k cos(2 pi (kx_k i + ky_k j) / n + theta_k) on an n x n
    grid (flat, row-major), wave numbers uniform in [1, kmax], A ~ U[0.5, 1],
    theta ~ U[0, 2 pi) (seeded).  Returns (v, [(kx, ky, A, theta), ...])."""
    rng = _rng(seed)
    modes = []
    i = np.arange(n, dtype=np.float64)
    v = np.zeros((n, n))
    for _ in range(count):
        kx, ky = (int(x) for x in rng.integers(1, kmax + 1, size=2))
        A, th = float(rng.uniform(0.5, 1.0)), float(rng.uniform(0.0, 2.0 * np.pi))
        ax = 2.0 * np.pi * kx * i / n + th
        ay = 2.0 * np.pi * ky * i / n
        # cos(ax + ay) = cos ax cos ay - sin ax sin ay, rows j, columns i
        v += A * (np.outer(np.cos(ay), np.cos(ax)) - np.outer(np.sin(ay), np.sin(ax)))
        modes.append((kx, ky, A, th))
    return v.ravel(), modes


def burgers_sines(n: int = 2048, nu: float = 1e-3, seed: int = 5, modes: int = 8) -> Problem:
    """Viscous Burgers u_t = nu Lap u - (1/2)(d_x + d_y)(u^2) on [0,1)^2.

    u0 = sum_k A_k sin(2 pi (m_k x + n_k y) + theta_k), m_k, n_k in {1..8},
    theta ~ U[0, 2 pi), A ~ U[0, 1], scaled to max|u0| = 1.  coef = (nu,).
    """
    dx = 1.0 / n
    rng = _rng(seed)
    m = rng.integers(1, 9, size=modes)
    k = rng.integers(1, 9, size=modes)
    th = rng.uniform(0.0, 2 * np.pi, size=modes)
    A = rng.uniform(0.0, 1.0, size=modes)
    x = np.arange(n) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.zeros((n, n))
    for j in range(modes):
        u += A[j] * np.sin(2 * np.pi * (m[j] * X + k[j] * Y) + th[j])
    u /= np.abs(u).max()
    return Problem("burgers", n, n, 1, dx, dx, (nu,), u.ravel().astype(np.float64), dx * dx / (4.0 * nu))


def batch_instances(count: int = 256, seed: int = 4, sizes=(128, 192, 256, 384, 512),
                    eps_range=(1e-4, 1e-2)):
    """Uneven ensemble of Allen-Cahn instances: n uniform over sizes, eps log-uniform.

    Instance i takes its noise from seed 4000 + i.  Returns a list of Problem.
    """
    rng = _rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    leps = rng.uniform(np.log(eps_range[0]), np.log(eps_range[1]), size=count)
    out = []
    for i in range(count):
        out.append(allen_cahn_noise(int(ns[i]), float(np.exp(leps[i])), seed=4000 + i))
    return out


def proposal_training_set(count: int, seed: int = 7, sizes=(32, 48, 64, 96, 128), hmult=(1.0, 100.0),
                          weights=None, families=("advdiff", "allencahn", "burgers")):
    """Seeded sweep of the training families of the learned proposal, drawn
    in turn with equal probability: advection-diffusion (grid Peclet
    log-uniform on [0.1, 4], Gaussian-bump input), Allen-Cahn (eps log-uniform
    on [1e-4, 1e-1], noise amplitude U[0.05, 1]) and viscous Burgers (nu
    log-uniform on [1e-4, 3e-2], eight random sine modes); n drawn from
    `sizes` (uniformly, or with the relative `weights`), h / h_cfl
    log-uniform on `hmult`.

    Returns a list of (problem, h, v) with v None for Allen-Cahn and Burgers
    (the caller uses h f(u) there) and the bump vector for
    advection-diffusion."""
    rng = _rng(seed)
    pw = None
    if weights is not None:
        pw = np.asarray(weights, dtype=np.float64)
        pw = pw / pw.sum()
    out = []
    for i in range(count):
        n = int(rng.choice(np.asarray(sizes), p=pw))
        hm = float(np.exp(rng.uniform(np.log(hmult[0]), np.log(hmult[1]))))
        fam = families[int(rng.integers(0, len(families)))]
        if fam == "advdiff":
            pe = float(np.exp(rng.uniform(np.log(0.1), np.log(4.0))))
            prob, v = advdiff_bump(n, nu=1.0, peclet=pe, seed=70000 + i)
        elif fam == "allencahn":
            eps = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-1))))
            amp = float(rng.uniform(0.05, 1.0))
            prob, v = allen_cahn_noise(n, eps=eps, seed=70000 + i, amp=amp), None
        else:
            nu = float(np.exp(rng.uniform(np.log(1e-4), np.log(3e-2))))
            prob, v = burgers_sines(n, nu=nu, seed=70000 + i), None
        out.append((prob, hm * prob.h_cfl, v))
    return out
