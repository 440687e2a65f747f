"""Pins of the learned-proposal oracle (features and the FP64 network): closed
forms of the features on special states, an independent loop-based feature
computation on tiny grids, the Gershgorin bound against the row sums of the
dense Jacobian assembled column by column from the oracle's own product
J e_q (every family, Neumann boundaries and grids so small that stencil
places coincide), central finite differences for the back-propagated
gradient, and the closed form of Adam's first step."""
import math

import numpy as np
import pytest

from oracle import features as F
from oracle import mlp
from oracle.operators import Operator
from workloads import (adr_neumann, advdiff_bump, allen_cahn_noise, brusselator_perturbed, burgers_sines,
                       diag_problem, gray_scott_spots)
from workloads.problems import Problem


def test_feature_count_and_pure_diffusion():
    p, _ = advdiff_bump(32, nu=2.0, peclet=0.0)
    h = 1e-3
    f = F.features(p, h, 1)
    assert f.shape == (16,)
    sigma = 2.0 * (1 / p.dx ** 2 + 1 / p.dy ** 2)
    # pure diffusion: |centre| = 2 sigma, the four neighbours add 2 sigma
    assert F.gershgorin(p) == pytest.approx(4.0 * sigma, rel=1e-15)
    assert f[0] == pytest.approx(math.log10(4.0 * h * sigma), rel=1e-15)
    assert f[1] == 0.25 and f[14] == pytest.approx(math.log10(4.0))
    # no advection, no reaction, no state
    assert np.all(f[[2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 13, 15]] == 0.0)
    assert f[12] == pytest.approx(math.log10(32 * 32) / 7)


def test_advection_rate_closed_form():
    p, _ = advdiff_bump(32, nu=1.0, peclet=1.0)
    sigma, A, r = F.scales(p)
    assert r is None
    assert A == pytest.approx(abs(p.coef[1]) / p.dx + abs(p.coef[2]) / p.dy)
    f = F.features(p, 3e-4, 2)
    assert f[2] == pytest.approx(math.log10(1 + A / sigma))
    assert f[5] == pytest.approx(math.log10(1 + 3e-4 * A))


def test_allen_cahn_constant_state():
    n, c, eps = 16, 0.3, 1e-2
    p = Problem("allencahn", n, n, 1, 2 / n, 2 / n, (eps,), np.full(n * n, c), (2 / n) ** 2 / (4 * eps))
    f = F.features(p, 0.5, 3)
    sigma = eps * 2 / (2 / n) ** 2
    r = 1 - 3 * c * c  # constant, positive
    assert f[3] == pytest.approx(math.log10(1 + r / sigma))
    assert f[4] == 0.0 and f[7] == 0.0
    assert f[6] == pytest.approx(math.log10(1 + 0.5 * r))
    assert f[8] == pytest.approx(1.0) and f[9] == pytest.approx(0.0, abs=1e-15)
    assert f[10] == pytest.approx(math.log10(1.3)) and f[11] == 0.0
    # |-2 sigma + r| + 2 sigma with 2 sigma > r
    assert F.gershgorin(p) == pytest.approx(4.0 * sigma - r, rel=1e-14)


def test_burgers_single_sine_closed_form():
    n = 64
    x = np.arange(n) / n
    X, _ = np.meshgrid(x, x)
    u = np.sin(2 * np.pi * X).ravel()
    p = Problem("burgers", n, n, 1, 1 / n, 1 / n, (1e-3,), u, (1 / n) ** 2 / 4e-3)
    sigma, A, r = F.scales(p)
    dx = 1 / n
    assert A == pytest.approx(2 / dx)  # max|u| = 1 at x = 1/4
    # r = -(d_x u) = -sin(2 pi dx)/dx cos(2 pi x): extremes at x = 0 and 1/2
    assert np.max(r) == pytest.approx(math.sin(2 * math.pi * dx) / dx, rel=1e-12)
    assert np.min(r) == pytest.approx(-math.sin(2 * math.pi * dx) / dx, rel=1e-12)
    _, _, umax, g = F.state_stats(p)
    assert umax == pytest.approx(1.0) and g == pytest.approx(math.sin(2 * math.pi * dx), rel=1e-12)


def _features_by_loops(p, h, l):
    """The feature definitions evaluated point by point (tiny grids only)."""
    nx, ny = p.nx, p.ny
    u = np.asarray(p.state, dtype=float)

    def at(i, j):
        if p.kind == "adr":  # Neumann: a boundary cell is its own ghost neighbour
            return u[min(max(j, 0), ny - 1) * nx + min(max(i, 0), nx - 1)]
        return u[(j % ny) * nx + (i % nx)]

    rs, gs, rows = [], [], []
    D0 = p.coef[0]
    for j in range(ny):
        for i in range(nx):
            # Gershgorin row of (i, j): entries per neighbour grid point, then |.|
            ent = {}

            def put(ii, jj, a):
                if p.kind == "adr":
                    key = (min(max(ii, 0), nx - 1), min(max(jj, 0), ny - 1))
                else:
                    key = (ii % nx, jj % ny)
                ent[key] = ent.get(key, 0.0) + a
            cx, cy = D0 / p.dx ** 2, D0 / p.dy ** 2
            if p.kind == "allencahn":
                put(i, j, -2 * (cx + cy) + 1 - 3 * at(i, j) ** 2)
                put(i - 1, j, cx), put(i + 1, j, cx), put(i, j - 1, cy), put(i, j + 1, cy)
            elif p.kind == "adr":
                c = at(i, j)
                be = p.coef[1]
                put(i, j, -2 * (cx + cy) + p.coef[2] * (3 * c - 3 * c * c - 0.5))
                put(i - 1, j, cx - be / (2 * p.dx)), put(i + 1, j, cx + be / (2 * p.dx))
                put(i, j - 1, cy - be / (2 * p.dy)), put(i, j + 1, cy + be / (2 * p.dy))
            else:  # burgers
                put(i, j, -2 * (cx + cy))
                put(i - 1, j, cx + at(i - 1, j) / (2 * p.dx)), put(i + 1, j, cx - at(i + 1, j) / (2 * p.dx))
                put(i, j - 1, cy + at(i, j - 1) / (2 * p.dy)), put(i, j + 1, cy - at(i, j + 1) / (2 * p.dy))
            rows.append(sum(abs(a) for a in ent.values()))
            if p.kind == "allencahn":
                rs.append(1 - 3 * at(i, j) ** 2)
            elif p.kind == "adr":
                c = at(i, j)
                rs.append(p.coef[2] * (3 * c - 3 * c * c - 0.5))
            else:  # burgers
                rs.append(-((at(i + 1, j) - at(i - 1, j)) / (2 * p.dx) + (at(i, j + 1) - at(i, j - 1)) / (2 * p.dy)))
            gs.append(math.hypot((at(i + 1, j) - at(i - 1, j)) / 2, (at(i, j + 1) - at(i, j - 1)) / 2))
    D = p.coef[0]
    sigma = D * (1 / p.dx ** 2 + 1 / p.dy ** 2)
    umax = max(abs(x) for x in u)
    A = 0.0
    if p.kind == "burgers":
        A = umax * (1 / p.dx + 1 / p.dy)
    elif p.kind == "adr":
        A = abs(p.coef[1]) * (1 / p.dx + 1 / p.dy)
    mean = sum(u) / len(u)
    std = math.sqrt(sum((x - mean) ** 2 for x in u) / len(u))
    rmax, rmin = max(rs), min(rs)
    G = max(rows)
    return [math.log10(h * G), l / 4, math.log10(1 + A / sigma), math.log10(1 + max(rmax, 0) / sigma),
            math.log10(1 + max(-rmin, 0) / sigma), math.log10(1 + h * A), math.log10(1 + h * max(rmax, 0)),
            math.log10(1 + h * max(-rmin, 0)), mean / umax, std / umax, math.log10(1 + umax),
            math.log10(1 + max(gs)), math.log10(nx * ny) / 7, math.log10(p.dx / p.dy),
            math.log10(G / sigma), 0.0]


@pytest.mark.parametrize("kind", ["allencahn", "burgers", "adr"])
def test_features_match_pointwise_loops(kind):
    if kind == "allencahn":
        p = allen_cahn_noise(12, eps=3e-3, seed=9)
    elif kind == "adr":
        p = adr_neumann(14, alpha=1e-2, amp=0.05, seed=9)
    else:
        p = burgers_sines(16, nu=2e-3, seed=9)
    h = 7.0 * p.h_cfl
    np.testing.assert_allclose(F.features(p, h, 2), _features_by_loops(p, h, 2), rtol=1e-13, atol=1e-15)


def test_targets():
    p = allen_cahn_noise(16, eps=1e-2, seed=2)
    G = F.gershgorin(p)
    t = F.targets(p, 0.5 * G, 8)
    assert t[0] == pytest.approx(math.log(0.5)) and t[1] == 3.0


def _dense_row_sum_max(p):
    """max_i sum_j |J_ij| with column q of J = the oracle's J e_q."""
    op = Operator(p)
    n = p.n
    J = np.empty((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        J[:, q] = op.jv(e)
    return float(np.max(np.sum(np.abs(J), axis=1)))


def _tiny(kind, nx, ny, seed):
    rng = np.random.default_rng(seed)
    dx, dy = 1.0 / nx, 1.3 / ny
    if kind == "advdiff":
        return Problem("advdiff", nx, ny, 1, dx, dy, (0.7, 9.0, -4.0), None, 1.0)
    if kind == "allencahn":
        return Problem("allencahn", nx, ny, 1, dx, dy, (2e-2,), rng.uniform(-1.2, 1.2, nx * ny), 1.0)
    if kind == "burgers":
        return Problem("burgers", nx, ny, 1, dx, dy, (3e-2,), rng.uniform(-2.0, 2.0, nx * ny), 1.0)
    if kind == "adr":
        return Problem("adr", nx, ny, 1, dx, dy, (1e-2, -10.0, 100.0), rng.uniform(-0.5, 1.5, nx * ny), 1.0)
    if kind == "brusselator":
        return Problem("brusselator", nx, ny, 2, dx, dy, (2e-3, 5e-3, 1.0, 3.0), rng.uniform(0.0, 4.0, 2 * nx * ny),
                       1.0)
    return Problem("grayscott", nx, ny, 2, dx, dy, (1e-3, 2e-3, 0.04, 0.06), rng.uniform(0.0, 1.0, 2 * nx * ny), 1.0)


@pytest.mark.parametrize("kind", ["advdiff", "allencahn", "burgers", "adr", "brusselator", "grayscott"])
@pytest.mark.parametrize("shape", [(7, 5), (2, 3), (1, 4)])
def test_gershgorin_equals_dense_row_sums(kind, shape):
    p = _tiny(kind, *shape, seed=3 + shape[0])
    assert F.gershgorin(p) == pytest.approx(_dense_row_sum_max(p), rel=1e-13)


def test_gershgorin_workload_states_and_diagonal():
    for p in (allen_cahn_noise(8, eps=1e-2, seed=4), burgers_sines(8, nu=2e-3, seed=4), adr_neumann(6, seed=4),
              brusselator_perturbed(6, seed=4), gray_scott_spots(8)):
        assert F.gershgorin(p) == pytest.approx(_dense_row_sum_max(p), rel=1e-13), p.kind
    d = diag_problem(50, -1e3, seed=5)
    assert F.gershgorin(d) == pytest.approx(float(np.max(np.abs(d.state))), rel=0)
    # the Gershgorin bound bounds the spectral radius
    for kind in ("burgers", "adr", "brusselator"):
        p = _tiny(kind, 6, 5, seed=11)
        op = Operator(p)
        J = np.stack([op.jv(np.eye(p.n)[q]) for q in range(p.n)], axis=1)
        assert np.max(np.abs(np.linalg.eigvals(J))) <= F.gershgorin(p) * (1 + 1e-12)


# ------------------------------------------------------------------ network
def _data(n=40, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16)) * 2 + 1
    T = rng.normal(size=(n, 2))
    mu, sd = X.mean(axis=0), X.std(axis=0) + 0.1
    tmu, tsd = T.mean(axis=0), T.std(axis=0) + 0.1
    return X, T, mu, sd, tmu, tsd


def test_param_layout_and_init():
    assert mlp.NPARAM == 64 * 16 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 5378
    th = mlp.init(6)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    assert np.all(b1 == 0) and np.all(b2 == 0) and np.all(b3 == 0)
    for W, (fo, fi) in ((W1, (64, 16)), (W2, (64, 64)), (W3, (2, 64))):
        a = math.sqrt(6 / (fo + fi))
        assert W.shape == (fo, fi) and np.max(np.abs(W)) <= a
        assert np.max(np.abs(W)) > 0.9 * a  # the draws fill the interval
    np.testing.assert_array_equal(mlp.pack(mlp.unpack(th)), th)
    np.testing.assert_array_equal(mlp.init(6), th)


def test_gradient_matches_central_differences():
    X, T, mu, sd, tmu, tsd = _data()
    th = mlp.init(6) + np.random.default_rng(1).normal(size=mlp.NPARAM) * 0.05
    L, g = mlp.grad(th, X, T, mu, sd, tmu, tsd)
    assert L == pytest.approx(mlp.loss(th, X, T, mu, sd, tmu, tsd), rel=1e-15)
    idx = np.random.default_rng(2).choice(mlp.NPARAM, 200, replace=False)
    idx = np.concatenate([idx, [0, 1023, 1024, 1087, 1088, 5183, 5184, 5311, 5376, 5377]])  # every block edge
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        step = 1e-6 * max(1.0, abs(th[i]))
        e[i] = step
        fd = (mlp.loss(th + e, X, T, mu, sd, tmu, tsd) - mlp.loss(th - e, X, T, mu, sd, tmu, tsd)) / (2 * step)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_zero_loss_at_exact_targets():
    X, _, mu, sd, tmu, tsd = _data()
    th = mlp.init(6)
    T = mlp.predict(th, X, mu, sd, tmu, tsd)
    L, g = mlp.grad(th, X, T, mu, sd, tmu, tsd)
    assert L == pytest.approx(0.0, abs=1e-28) and np.max(np.abs(g)) <= 1e-14


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    th, g = rng.normal(size=50), rng.normal(size=50)
    th1, m, v = mlp.adam_step(th, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # after one step the bias-corrected moments are g and g^2
    np.testing.assert_allclose(th - th1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g) and np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_descends_on_a_small_fit():
    X, T, mu, sd, tmu, tsd = _data(64, seed=8)
    th = mlp.init(6)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = mlp.loss(th, X, T, mu, sd, tmu, tsd)
    for t in range(1, 201):
        _, g = mlp.grad(th, X, T, mu, sd, tmu, tsd)
        th, m, v = mlp.adam_step(th, m, v, g, t, 3e-3)
    assert mlp.loss(th, X, T, mu, sd, tmu, tsd) < 0.2 * L0
