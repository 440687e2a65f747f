"""Pins of the oracle's stencils and power iteration against independent
constructions: sparse Kronecker assembly, finite differences of the RHS,
Fourier modes, exact fixed points and dense eigenvalues."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.exact import advdiff_symbol
from oracle.operators import Operator
from oracle.power import power_iteration
from workloads import (advdiff_bump, allen_cahn_noise, brusselator_perturbed,
                       burgers_sines, gray_scott_spots)
from workloads.problems import Problem


def _d2(n, h):
    e = np.ones(n)
    D = sp.diags([e[:-1], -2 * e, e[:-1]], [-1, 0, 1], shape=(n, n)).tolil()
    D[0, n - 1] = 1.0
    D[n - 1, 0] = 1.0
    return (D / (h * h)).tocsr()


def _d1(n, h):
    e = np.ones(n)
    D = sp.diags([-e[:-1], e[:-1]], [-1, 1], shape=(n, n)).tolil()
    D[0, n - 1] = -1.0
    D[n - 1, 0] = 1.0
    return (D / (2 * h)).tocsr()


def _d2n(n, h):
    # homogeneous Neumann, cell-centred: ghost u_{-1} = u_0, u_n = u_{n-1}
    e = np.ones(n)
    d = -2 * e
    d[0] = d[-1] = -1.0
    return (sp.diags([e[:-1], d, e[:-1]], [-1, 0, 1], shape=(n, n)) / (h * h)).tocsr()


def _d1n(n, h):
    e = np.ones(n)
    d = np.zeros(n)
    d[0], d[-1] = -1.0, 1.0
    return (sp.diags([-e[:-1], d, e[:-1]], [-1, 0, 1], shape=(n, n)) / (2 * h)).tocsr()


def _kron_ops(nx, ny, dx, dy):
    Ix, Iy = sp.identity(nx), sp.identity(ny)
    lap = sp.kron(Iy, _d2(nx, dx)) + sp.kron(_d2(ny, dy), Ix)
    dxo = sp.kron(Iy, _d1(nx, dx))
    dyo = sp.kron(_d1(ny, dy), Ix)
    return lap.toarray(), dxo.toarray(), dyo.toarray()


def _small(kind, nx=7, ny=5):
    rng = np.random.default_rng(11)
    dx, dy = 0.13, 0.21
    if kind == "advdiff":
        return Problem(kind, nx, ny, 1, dx, dy, (0.7, 1.3, -0.4), None, 1.0)
    if kind == "allencahn":
        return Problem(kind, nx, ny, 1, dx, dy, (0.05,), rng.uniform(-1, 1, nx * ny), 1.0)
    if kind == "burgers":
        return Problem(kind, nx, ny, 1, dx, dy, (0.02,), rng.uniform(-1, 1, nx * ny), 1.0)
    if kind == "brusselator":
        return Problem(kind, nx, ny, 2, dx, dy, (0.03, 0.011, 1.0, 3.0),
                       rng.uniform(0.5, 3.5, 2 * nx * ny), 1.0)
    if kind == "grayscott":
        return Problem(kind, nx, ny, 2, dx, dy, (0.02, 0.007, 0.04, 0.06),
                       rng.uniform(0.0, 1.0, 2 * nx * ny), 1.0)
    if kind == "adr":
        return Problem(kind, nx, ny, 1, dx, dy, (0.03, -1.7, 9.0), rng.uniform(-0.2, 1.2, nx * ny), 1.0)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["advdiff", "allencahn", "burgers", "brusselator", "grayscott", "adr"])
def test_jacobian_matches_kronecker_assembly(kind):
    p = _small(kind)
    op = Operator(p)
    J = op.dense()
    lap, dxo, dyo = _kron_ops(p.nx, p.ny, p.dx, p.dy)
    if kind == "advdiff":
        nu, ax, ay = p.coef
        ref = nu * lap - ax * dxo - ay * dyo
    elif kind == "allencahn":
        (eps,) = p.coef
        ref = eps * lap + np.diag(1 - 3 * p.state ** 2)
    elif kind == "burgers":
        (nu,) = p.coef
        ref = nu * lap - (dxo + dyo) @ np.diag(p.state)
    elif kind == "brusselator":
        Du, Dv, a, b = p.coef
        U, V = p.state[0::2], p.state[1::2]
        n = p.nx * p.ny
        blk = np.zeros((2 * n, 2 * n))
        blk[0::2, 0::2] = Du * lap + np.diag(-(b + 1) + 2 * U * V)
        blk[0::2, 1::2] = np.diag(U * U)
        blk[1::2, 0::2] = np.diag(b - 2 * U * V)
        blk[1::2, 1::2] = Dv * lap - np.diag(U * U)
        ref = blk
    elif kind == "adr":
        # Neumann boundaries: Kronecker sums of the 1D Neumann differences
        alpha, beta, rate = p.coef
        Ix, Iy = sp.identity(p.nx), sp.identity(p.ny)
        lapn = (sp.kron(Iy, _d2n(p.nx, p.dx)) + sp.kron(_d2n(p.ny, p.dy), Ix)).toarray()
        grad = (sp.kron(Iy, _d1n(p.nx, p.dx)) + sp.kron(_d1n(p.ny, p.dy), Ix)).toarray()
        u = p.state
        ref = alpha * lapn + beta * grad + np.diag(rate * (-3 * u * u + 3 * u - 0.5))
    else:  # Gray-Scott: partial derivatives of -u v^2 + a(1 - u) and u v^2 - (a + b) v
        a1, a2, a, b = p.coef
        U, V = p.state[0::2], p.state[1::2]
        n = p.nx * p.ny
        blk = np.zeros((2 * n, 2 * n))
        blk[0::2, 0::2] = a1 * lap + np.diag(-V * V - a)
        blk[0::2, 1::2] = np.diag(-2 * U * V)
        blk[1::2, 0::2] = np.diag(V * V)
        blk[1::2, 1::2] = a2 * lap + np.diag(2 * U * V - (a + b))
        ref = blk
    assert np.max(np.abs(J - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("kind", ["allencahn", "burgers", "brusselator", "grayscott", "adr"])
def test_jacobian_is_derivative_of_rhs(kind):
    p = _small(kind)
    op = Operator(p)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(p.n)
    jv = op.jv(v)
    errs = []
    for eps in [1e-2, 5e-3]:
        fd = (op.rhs(p.state + eps * v) - op.rhs(p.state - eps * v)) / (2 * eps)
        errs.append(np.linalg.norm(fd - jv) / np.linalg.norm(jv))
    # central differences: error O(eps^2) (exact 0 for quadratic RHS)
    assert errs[0] < 1e-3
    assert errs[1] <= errs[0] / 3.5 or errs[1] < 1e-12


def test_allen_cahn_jacobian_symmetric():
    J = Operator(_small("allencahn")).dense()
    assert np.max(np.abs(J - J.T)) <= 1e-13 * np.max(np.abs(J))


def test_brusselator_steady_state_is_fixed_point():
    p = _small("brusselator")
    a, b = p.coef[2], p.coef[3]
    st = np.empty(2 * p.nx * p.ny)
    st[0::2], st[1::2] = a, b / a
    assert np.max(np.abs(Operator(p).rhs(st))) <= 1e-15


def test_gray_scott_trivial_state_is_fixed_point():
    # (u, v) = (1, 0): no reaction (u v^2 = 0, a(1 - u) = 0, (a + b) v = 0) and no diffusion
    p = _small("grayscott")
    st = np.empty(2 * p.nx * p.ny)
    st[0::2], st[1::2] = 1.0, 0.0
    assert np.max(np.abs(Operator(p).rhs(st))) == 0.0


def test_adr_constant_roots_are_fixed_points():
    # u = 0, 1/2, 1 are roots of the reaction; Neumann differences of a constant vanish
    p = _small("adr")
    op = Operator(p)
    for c in (0.0, 0.5, 1.0):
        assert np.max(np.abs(op.rhs(np.full(p.n, c)))) == 0.0


def test_adr_neumann_conserves_mass_without_advection_and_reaction():
    # with ghost = boundary cell, the Neumann Laplacian's columns sum to zero
    p = _small("adr")
    p.coef = (0.03, 0.0, 0.0)
    v = np.random.default_rng(4).standard_normal(p.n)
    jv = Operator(p).jv(v)
    assert abs(jv.sum()) <= 1e-12 * np.abs(jv).sum()


def test_neumann_diffusion_dct_modes_are_eigenvectors():
    # J cos(pi kx (i + 1/2)/nx) cos(pi ky (j + 1/2)/ny) = lam[ky, kx] (same mode):
    # pins the Neumann boundary rows against the closed form used by the action pins
    from oracle.exact import neumann_diffusion_eigs
    p = _small("adr", 8, 6)
    p.coef = (0.03, 0.0, 0.0)
    op = Operator(p)
    lam = neumann_diffusion_eigs(p.nx, p.ny, p.dx, p.dy, 0.03)
    I, Jg = np.meshgrid(np.arange(p.nx), np.arange(p.ny), indexing="xy")
    for a in range(p.ny):
        for b in range(p.nx):
            mode = (np.cos(np.pi * b * (I + 0.5) / p.nx) * np.cos(np.pi * a * (Jg + 0.5) / p.ny)).ravel()
            assert np.allclose(op.jv(mode), lam[a, b] * mode, atol=1e-10 * max(1.0, abs(lam[a, b])))


def test_advdiff_fourier_modes_are_eigenvectors():
    # J e^{i(tx i + ty j)} = sigma(tx, ty) e^{i(...)}: pins the stencil's
    # orientation and signs together with the symbol used by the closed form
    p = _small("advdiff", 8, 6)
    op = Operator(p)
    sig = advdiff_symbol(p.nx, p.ny, p.dx, p.dy, *p.coef)
    kx = 2 * np.pi * np.fft.fftfreq(p.nx)
    ky = 2 * np.pi * np.fft.fftfreq(p.ny)
    I, Jg = np.meshgrid(np.arange(p.nx), np.arange(p.ny), indexing="xy")
    for a in range(p.ny):
        for b in range(p.nx):
            mode = np.exp(1j * (kx[b] * I + ky[a] * Jg)).ravel()
            got = op.jv(mode.real) + 1j * op.jv(mode.imag)
            assert np.allclose(got, sig[a, b] * mode, atol=1e-10)


def test_workload_shapes_and_seeds():
    p, v = advdiff_bump()
    assert p.n == 1024 and v.shape == (1024,)
    assert abs(p.coef[1] * p.dx / p.coef[0] - 1.0) < 1e-15  # grid Peclet 1
    ac = allen_cahn_noise(64, seed=2)
    assert np.all(np.abs(ac.state) <= 0.1)
    assert np.array_equal(ac.state, allen_cahn_noise(64, seed=2).state)
    br = brusselator_perturbed(16)
    assert np.all(np.abs(br.state[0::2] - 1) <= 1e-2) and np.all(np.abs(br.state[1::2] - 3) <= 1e-2)
    bu = burgers_sines(64)
    assert abs(np.abs(bu.state).max() - 1.0) < 1e-15
    gs = gray_scott_spots(64)
    assert gs.ncomp == 2 and gs.n == 2 * 64 * 64
    assert 0.0 <= gs.state[0::2].min() and gs.state[0::2].max() <= 1.0 and 0.9 < gs.state[1::2].max() <= 1.0


# ------------------------------------------------------------ power iteration
def test_power_iteration_below_spectral_radius_normal():
    # normal J: ||J x|| / ||x|| <= rho(J), and the estimate approaches rho
    p = allen_cahn_noise(16, eps=1e-2, seed=9)
    op = Operator(p)
    rho = np.max(np.abs(np.linalg.eigvalsh(op.dense())))
    lam20 = power_iteration(op.jv, p.n, 20)
    lam_long = power_iteration(op.jv, p.n, 3000)
    assert lam20 <= rho * (1 + 1e-14)
    assert lam20 >= 0.9 * rho
    assert abs(lam_long - rho) <= 1e-6 * rho
    assert 1.25 * lam20 >= rho


def test_power_iteration_advdiff_config():
    p, _ = advdiff_bump()
    op = Operator(p)
    rho = np.max(np.abs(advdiff_symbol(p.nx, p.ny, p.dx, p.dy, *p.coef)))
    lam = power_iteration(op.jv, p.n, 20)
    assert abs(rho - 8192.0) < 1e-9  # 8 nu / dx^2 at the Nyquist mode
    assert 0.9 * rho <= lam <= rho * (1 + 1e-14)
    assert 1.25 * lam >= rho


def test_power_iteration_diagonal_dominant():
    lam = np.array([-1.0, -2.0, -3.0, -10.0])
    est = power_iteration(lambda x: lam * x, 4, 200)
    assert abs(est - 10.0) < 1e-12
    gersh = np.max(np.abs(lam))
    assert est <= gersh * (1 + 1e-15)
