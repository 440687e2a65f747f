"""Pins of the oracle's Leja action against closed forms (elementwise phi for a
diagonal J, Fourier diagonalisation, dense Pade expm of the Sec. 2.1 augmented
matrix), the paper's qualitative claims, the substep identity and the
rejection rules; and of the stage driver against e^{hJ} and its order."""
from dataclasses import replace
from fractions import Fraction

import numpy as np
import pytest

import oracle.leja as leja
from oracle.exact import (advdiff_symbol, dct_closed_form, diag_closed_form, fourier_closed_form,
                          neumann_diffusion_eigs, phi_dense)
from oracle.integrators import rk_reference, step
from oracle.leja import Options, phi_action, phi_vertical
from oracle.operators import Operator
from oracle.phi import phi
from workloads import (adr_neumann, advdiff_bump, allen_cahn_noise, brusselator_perturbed, diag_problem,
                       gray_scott_spots)
from workloads.problems import Problem


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def cfg1():
    p, v = advdiff_bump()
    op = Operator(p)
    sig = advdiff_symbol(p.nx, p.ny, p.dx, p.dy, *p.coef)
    return p, v, op, sig


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_diagonal_closed_form(l):
    p = diag_problem(400, -500.0, seed=3)
    op = Operator(p)
    v = np.random.default_rng(l).uniform(-1, 1, 400)
    h = 0.2
    ref = diag_closed_form(p.state, v, l, h, phi)
    w, st = phi_action(op, v, l, h, 1e-14)
    assert st.converged and rel(w, ref) <= 1e-12
    w, st = phi_action(op, v, l, h, 1e-10)
    assert rel(w, ref) <= 1e-9


@pytest.mark.parametrize("l", [1, 2])
def test_fourier_closed_form_config1(cfg1, l):
    p, v, op, sig = cfg1
    h = 10 * p.h_cfl
    ref = fourier_closed_form(sig, v, l, h)
    w, st = phi_action(op, v, l, h, 1e-10)
    assert rel(w, ref) <= 1e-9
    w, st = phi_action(op, v, l, h, 1e-14)
    assert rel(w, ref) <= 1e-12


def test_fourier_matches_dense_pade(cfg1):
    p, v, op, sig = cfg1
    h = 10 * p.h_cfl
    ref_f = fourier_closed_form(sig, v, 1, h)
    ref_d = phi_dense(h * op.dense(), v, 1)
    assert rel(ref_f, ref_d) <= 1e-13


@pytest.mark.parametrize("l", [1, 2])
def test_dct_closed_form_neumann_diffusion(l):
    # pure diffusion with homogeneous Neumann boundaries (cell-centred): the
    # 2D DCT-II diagonalises J
    nx, ny, dx, dy, alpha = 32, 24, 1 / 32, 1 / 24, 1e-2
    p = Problem("adr", nx, ny, 1, dx, dy, (alpha, 0.0, 0.0), np.zeros(nx * ny), dx * dx / (4 * alpha))
    op = Operator(p)
    v = np.random.default_rng(3).uniform(0, 1, p.n)
    h = 10 * p.h_cfl
    ref = dct_closed_form(neumann_diffusion_eigs(nx, ny, dx, dy, alpha), v, l, h)
    w, st = phi_action(op, v, l, h, 1e-10)
    assert st.converged and rel(w, ref) <= 1e-9
    w, st = phi_action(op, v, l, h, 1e-14)
    assert st.converged and rel(w, ref) <= 1e-12


@pytest.mark.parametrize("kind", ["allencahn", "brusselator", "burgers", "grayscott", "adr"])
@pytest.mark.parametrize("l", [0, 1, 3])
def test_dense_pade_small_grids(kind, l):
    if kind == "allencahn":
        p = allen_cahn_noise(16, eps=1e-2, seed=8)
        p.state = p.state * 8  # reach the nonlinear range |u| <= 0.8
    elif kind == "brusselator":
        # diffusion-dominated, as at 1024^2 with D = 2e-3: the reaction's unstable
        # pair (Re = 1/2) then sits just beyond the right end of the interval
        p = brusselator_perturbed(12, D=0.1, seed=8, amp=0.3)
    elif kind == "grayscott":
        p = gray_scott_spots(12, a1=2e-2, a2=1e-2, amp=0.05)
    elif kind == "adr":
        # grid Peclet |beta| dx / alpha < 2 (real spectrum), strong reaction
        p = adr_neumann(12, alpha=0.1, beta=-1.0, rate=100.0, amp=0.05)
    else:
        # grid Peclet ~1.25: diffusion-dominated like the 2048^2 workload
        p = Problem("burgers", 16, 16, 1, 1 / 16, 1 / 16, (5e-2,),
                    np.sin(2 * np.pi * np.arange(256) / 256 * 3), (1 / 16) ** 2 / 0.2)
    op = Operator(p)
    v = np.random.default_rng(1).uniform(-1, 1, p.n)
    h = 10 * p.h_cfl
    ref = phi_dense(h * op.dense(), v, l)
    w, st = phi_action(op, v, l, h, 1e-14)
    assert st.converged and rel(w, ref) <= 1e-12
    w, st = phi_action(op, v, l, h, 1e-10)
    assert rel(w, ref) <= 1e-9


# ------------------------------------------------- the paper's qualitative claims
def test_more_points_for_larger_steps(cfg1):
    # Sec. 2.2: larger step sizes need more Leja points
    p, v, op, _ = cfg1
    ms = [phi_action(op, v, 1, k * p.h_cfl, 1e-10)[1].m_star[0] for k in (1, 3, 10, 30)]
    assert ms == sorted(ms) and ms[0] < ms[-1]


def test_higher_phi_converges_faster():
    # Appendix A: higher-order phi functions converge faster
    p = allen_cahn_noise(64, eps=1e-3, seed=2)
    op = Operator(p)
    v = 10 * p.h_cfl * op.rhs(p.state)
    ms = [phi_action(op, v, l, 30 * p.h_cfl, 1e-10)[1].m_star[0] for l in (1, 2, 3)]
    assert ms[2] <= ms[1] <= ms[0]


def test_vertical_shares_basis_and_saves_work():
    # Sec. 4: phi_1 at 1/8, 1/9 and 1 on the same vector cost about one action
    p = allen_cahn_noise(64, eps=1e-3, seed=2)
    op = Operator(p)
    h = 10 * p.h_cfl
    v = h * op.rhs(p.state)
    As = [1 / 8, 1 / 9, 1.0]
    lam = leja.power_iteration(op.jv, p.n, 20)
    o = Options(bound=lam)
    ws, st = phi_vertical(op, v, [1, 1, 1], As, h, 1e-10, o)
    single = [phi_vertical(op, v, [1], [a], h, 1e-10, o) for a in As]
    for k in range(3):
        # identical arithmetic on the shared basis: bit-identical results
        assert np.array_equal(ws[k], single[k][0][0])
        assert st.m_star[k] == single[k][1].m_star[0]
    # smaller coefficient -> fewer points (Sec. 4, EPIRK4s3 vs EPIRK4s3A)
    assert st.m_star[0] <= st.m_star[2] and st.m_star[1] <= st.m_star[2]
    assert st.iters_total == max(st.m_star) < sum(s[1].iters_total for s in single)


# ---------------------------------------------------------------- substepping
@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_substep_identity_diagonal(l):
    p = diag_problem(300, -400.0, seed=4)
    op = Operator(p)
    v = np.random.default_rng(2).uniform(-1, 1, 300)
    h = 0.25
    ref = diag_closed_form(p.state, v, l, h, phi)
    for s in (2, 4, 8):
        w, st = phi_action(op, v, l, h, 1e-14, Options(substeps=s))
        assert st.converged and st.substeps == [s]
        assert rel(w, ref) <= 1e-12, (l, s)


def test_substep_invariance_advdiff(cfg1):
    p, v, op, sig = cfg1
    h = 10 * p.h_cfl
    base, _ = phi_action(op, v, 2, h, 1e-10)
    for s in (2, 4, 8):
        w, st = phi_action(op, v, 2, h, 1e-10, Options(substeps=s))
        assert rel(w, base) <= s * 10 * 1e-10


def test_rejection_then_substeps_config1_100cfl(cfg1):
    p, v, op, sig = cfg1
    h = 100 * p.h_cfl
    w, st = phi_action(op, v, 1, h, 1e-10)
    assert st.rejections >= 1 and st.substeps[0] >= 2 and st.converged
    assert rel(w, fourier_closed_form(sig, v, 1, h)) <= 1e-8


def test_forced_small_max_points_triggers_substepping(cfg1):
    p, v, op, sig = cfg1
    h = 10 * p.h_cfl
    w, st = phi_action(op, v, 1, h, 1e-10, Options(max_points=12))
    assert st.rejections >= 1 and st.substeps[0] > 1 and st.converged
    assert rel(w, fourier_closed_form(sig, v, 1, h)) <= 1e-8


def test_substeps_reach_dense_pade_on_burgers():
    # advection-heavier Burgers: s = 1 is rejected, substeps recover the Pade result
    p = Problem("burgers", 16, 16, 1, 1 / 16, 1 / 16, (2e-2,),
                np.sin(2 * np.pi * np.arange(256) / 256 * 3), (1 / 16) ** 2 / 0.08)
    op = Operator(p)
    v = np.random.default_rng(1).uniform(-1, 1, p.n)
    h = 10 * p.h_cfl
    w, st = phi_action(op, v, 1, h, 1e-10)
    assert st.converged and st.rejections >= 1 and st.substeps[0] >= 2
    assert rel(w, phi_dense(h * op.dense(), v, 1)) <= 1e-9


def test_no_substeps_allowed_reports_failure(cfg1):
    p, v, op, _ = cfg1
    w, st = phi_action(op, v, 1, 100 * p.h_cfl, 1e-10, Options(max_substeps=1))
    assert not st.converged


def test_zero_vector_and_nonfinite(cfg1):
    p, v, op, _ = cfg1
    w, st = phi_action(op, np.zeros(p.n), 1, 10 * p.h_cfl, 1e-10)
    assert st.converged and np.all(w == 0) and st.m_star == [0]
    bad = v.copy()
    bad[17] = np.nan
    w, st = phi_action(op, bad, 1, 10 * p.h_cfl, 1e-10, Options(max_substeps=2))
    assert not st.converged


# ------------------------------------------------------- hump rejection (C.7)
def _term_ratios(lam, v, l, T, c, gamma, xi, M):
    """e_m / (||v|| max_j |f_j|), m = 1..M, for a diagonal J = diag(lam), with
    the Newton basis in closed form, y_m = prod_{j<m} ((lam - c)/gamma - xi_j) v
    elementwise (nothing of the oracle's recurrence).  Two sets of
    coefficients: the exact divided differences of phi_l at the scaled nodes
    (60 digits, phi_l from its Sec. 1 definition), and the FP64 table of
    oracle.divdiff on oracle.phi's node values (each pinned on its own
    against 50-digit values); at high orders the FP64 table is rounding
    noise amplified, so only the same FP64 node values reproduce it."""
    import mpmath as mp
    from oracle.divdiff import divided_differences
    mp.mp.dps = 60

    def phi_mp(z):
        if z == 0:
            return 1 / mp.factorial(l)
        s = mp.e ** z
        for k in range(l):
            s -= z ** k / mp.factorial(k)
        return s / z ** l

    f = [phi_mp(mp.mpf(T) * (mp.mpf(c) + mp.mpf(gamma) * mp.mpf(x))) for x in xi[:M + 1]]
    d = list(f)
    for k in range(1, M + 1):
        for j in range(M, k - 1, -1):
            d[j] = (d[j] - d[j - 1]) / (mp.mpf(xi[j]) - mp.mpf(xi[j - k]))
    f64 = [phi(l, T * (c + gamma * x)) for x in xi[:M + 1]]
    d64 = divided_differences(f64, xi[:M + 1])
    scale = np.linalg.norm(v) * max(abs(x) for x in f64)
    q = (np.asarray(lam) - c) / gamma
    y = np.array(v, dtype=np.float64)
    exact, fp64 = [], []
    for m in range(1, M + 1):
        y = (q - xi[m - 1]) * y
        ny = np.linalg.norm(y)
        exact.append(abs(float(d[m])) * ny / scale)
        fp64.append(abs(d64[m]) * ny / scale)
    return np.array(exact), np.array(fp64)


@pytest.mark.parametrize("l,hump", [(0, 1e4), (1, 1e4), (3, 1e2)])
def test_hump_rejection_index(l, hump, xi101):
    """Sec. 2.2, last paragraph: with many Leja points the divided differences
    are round-off prone, and an expansion that does not settle is rejected.
    With the bound at 0.6 of the true spectral radius the diagonal operator's
    eigenvalues near -500 map to -4.4 on the Leja scale and the Newton basis
    grows geometrically.  In exact arithmetic the coefficients still fall
    faster (every term ratio stays below 1), but the FP64 rounding of the
    table is amplified by the basis and the terms pass hump_max ||v|| max|f|
    (C.7) long before max_points.  The oracle must reject at exactly the
    first m at which the term ratio crosses hump_max (the crossing is by
    more than 1 % either side, far beyond the rounding of the basis, so no
    rounding order decides it), and
    with no hump limit the same run must go on to max_points."""
    p = diag_problem(400, -500.0, seed=3)
    op = Operator(p)
    v = np.random.default_rng(5).uniform(-1, 1, 400)
    lam, h = 300.0, 0.02
    c, gamma = leja.interval(lam, 1.25)
    exact, fp64 = _term_ratios(p.state, v, l, h, c, gamma, xi101, 100)
    assert np.all(exact < 1.0)
    assert np.any(fp64 > hump)
    expect = int(np.argmax(fp64 > hump)) + 1
    assert fp64[expect - 1] > 1.01 * hump and np.all(fp64[:expect - 1] < hump / 1.01)
    r = leja.newton_recurrence(op.jv, v, [l], [1.0], h, c, gamma, 1e-10, Options(hump_max=hump))
    assert r.reason == ["hump"] and not r.converged[0] and r.iters == expect
    r = leja.newton_recurrence(op.jv, v, [l], [1.0], h, c, gamma, 1e-10, Options(hump_max=1e300))
    assert r.reason == ["maxpts"] and r.iters == 100


@pytest.mark.parametrize("l", [0, 1, 3])
def test_hump_rejection_then_substeps_reach_closed_form(l):
    """After a hump rejection the action is redone with s = 2, 4, ...; the
    substeps shrink tau gamma until the terms decay faster than the basis
    grows, and the result is phi_l(hJ)v within 10 s tol."""
    p = diag_problem(400, -500.0, seed=3)
    op = Operator(p)
    v = np.random.default_rng(5).uniform(-1, 1, 400)
    h = 0.02
    w, st = phi_action(op, v, l, h, 1e-10, Options(bound=300.0))
    assert st.converged and st.rejections >= 1 and st.substeps[0] >= 2
    ref = diag_closed_form(p.state, v, l, h, phi)
    assert rel(w, ref) <= 10 * st.substeps[0] * 1e-10


@pytest.mark.parametrize("l", [0, 1, 3])
def test_small_hump_limit_forces_substeps(l):
    """With the right bound the first term of an expansion at a large
    tau gamma is about 0.45 ||v|| max|f|, so hump_max = 0.2 rejects at m = 1
    until the substeps make tau gamma small: s = 8 here (the first term then
    falls to 0.45 (1 - e^{-4 tau gamma}) ||v|| max|f| ~ 0.18), and the result
    is phi_l(hJ)v within 10 s tol."""
    p = diag_problem(400, -500.0, seed=3)
    op = Operator(p)
    v = np.random.default_rng(5).uniform(-1, 1, 400)
    h = 0.0064
    w, st = phi_action(op, v, l, h, 1e-10, Options(bound=500.0, hump_max=0.2))
    assert st.converged and st.substeps == [8] and st.rejections == 3
    assert rel(w, diag_closed_form(p.state, v, l, h, phi)) <= 80 * 1e-10
    w1, st1 = phi_action(op, v, l, h, 1e-10, Options(bound=500.0))
    assert st1.substeps == [1] and st1.rejections == 0


# ------------------------------------------------------------ planted mistakes
def test_planted_mistakes_are_caught(cfg1, monkeypatch):
    """Each plausible slip in the oracle makes a pin fail: the Fourier closed
    form for slips that change the result, the point count for slips in the
    interval map (a Leja expansion of an entire function still converges on a
    badly placed interval, only at a different cost)."""
    p, v, op, sig = cfg1
    h = 10 * p.h_cfl
    ref = fourier_closed_form(sig, v, 1, h)

    def run_with(patch):
        with monkeypatch.context() as mp_:
            patch(mp_)
            leja._XI_CACHE.clear()
            try:
                w, st = phi_action(op, v, 1, h, 1e-10)
                return rel(w, ref), st
            except Exception:
                return np.inf, None
            finally:
                leja._XI_CACHE.clear()

    err0, st0 = run_with(lambda m: None)
    assert err0 <= 1e-9 and st0.m_star == [28] and st0.rejections == 0
    # gamma an eighth instead of a quarter of the interval length
    _, st = run_with(lambda m: m.setattr(leja, "interval", lambda lam, s: (-0.5 * s * lam, 0.125 * s * lam)))
    assert st is None or st.m_star != st0.m_star or st.rejections > 0
    # wrong sign of the shift c
    err, st = run_with(lambda m: m.setattr(leja, "interval", lambda lam, s: (0.5 * s * lam, 0.25 * s * lam)))
    assert err > 1e-6 or st is None or st.iters_total > 3 * st0.iters_total
    # a dropped divided-difference order (coefficients shifted by one)
    orig = leja.divided_differences
    err, _ = run_with(lambda m: m.setattr(leja, "divided_differences",
                                          lambda f, xi: np.concatenate([orig(f, xi)[:5], orig(f, xi)[6:], [0.0]])))
    assert err > 1e-6
    # a moved node used consistently is still a valid interpolation: cost changes
    _, st = run_with(lambda m: m.setattr(leja, "leja_points", lambda n: _moved_node(orig_points(n))))
    assert st is None or st.m_star != st0.m_star or st.err != st0.err
    # coefficients taken at nodes one index off from the recurrence's nodes
    xi = orig_points(102)

    def shifted(l, a, tau, c, gamma, npts):
        f = [phi(l, a * tau * (c + gamma * x)) for x in xi[1:npts + 1]]
        return orig(f, xi[1:npts + 1]), max(abs(x) for x in f)

    err, _ = run_with(lambda m: m.setattr(leja, "coefficients", shifted))
    assert err > 1e-6
    # phi_l index off by one
    err, _ = run_with(lambda m: m.setattr(leja, "phi", lambda l, z: phi(l + 1, z)))
    assert err > 1e-6


def _moved_node(x):
    x = x.copy()
    x[7] += 1e-3
    return x


def orig_points(n):
    from oracle.points import leja_points
    return leja_points(n)


# --------------------------------------------------------------- stage driver
@pytest.mark.parametrize("scheme", ["EXPRB2", "EXPRB43", "EXPRB43_U3", "EPIRK4S3", "EPIRK4S3A"])
def test_linear_problem_every_scheme_is_exact_exponential(cfg1, scheme):
    # f(u) = J u  =>  R = 0 and u + h phi_1(hJ) J u = e^{hJ} u
    p, v, op, sig = cfg1
    lin = Operator(p, state=v)
    h = 10 * p.h_cfl
    u_out, err, _ = step(lin, scheme, h, 1e-12)
    ref = fourier_closed_form(sig, v, 0, h)
    assert rel(u_out, ref) <= 1e-10
    if err is not None:
        assert np.linalg.norm(err) <= 1e-10 * np.linalg.norm(ref)


def test_printed_coefficients_satisfy_stiff_order_conditions():
    # With R(U_i) = O(c_i^2) the weights b_i(z) must give sum b_i c_i^2 = 2 phi_3
    # (order 3) and sum b_i c_i^3 = 6 phi_4 (order 4).  Weights as (phi_3, phi_4)
    # coefficient pairs, from the equations of Sec. 5.1, 5.2 and 5.4.
    F = Fraction
    epirk = {F(1, 8): (F(1892) - 2 * F(1458), F(-42336) + 2 * F(34992)), F(1, 9): (F(1458), F(-34992))}
    epirk_a = {F(1, 2): (F(32), F(-144)), F(2, 3): (F(-27, 2), F(81))}
    exprb = {F(1, 2): (F(16), F(-48)), F(1): (F(-2), F(12))}
    for tab in (epirk, epirk_a, exprb):
        c2 = [sum(b[i] * c ** 2 for c, b in tab.items()) for i in (0, 1)]
        c3 = [sum(b[i] * c ** 3 for c, b in tab.items()) for i in (0, 1)]
        assert c2 == [2, 0] and c3 == [0, 6]


@pytest.mark.slow
def test_observed_order_allen_cahn():
    # local error of one step vs a fine RK4 reference shrinks like h^(p+1)
    n = 12
    x = (np.arange(n) + 0.5) / n * 2 - 1
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = (0.5 + 0.3 * np.cos(np.pi * X) * np.sin(np.pi * Y)).ravel()
    base = Problem("allencahn", n, n, 1, 2 / n, 2 / n, (0.02,), u0, 1.0)
    mk = lambda u: Operator(base, state=u)  # noqa: E731
    expect = {"EXPRB2": 3, "EXPRB43_U3": 4, "EXPRB43": 5, "EPIRK4S3": 5, "EPIRK4S3A": 5}
    for scheme, order in expect.items():
        errs = []
        hs = [0.4, 0.2, 0.1]
        for h in hs:
            u1, _, _ = step(mk(u0), scheme, h, 1e-14)
            ref = rk_reference(mk, u0, h, 400)
            errs.append(np.linalg.norm(u1 - ref))
        rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert rates[-1] >= order - 0.6, (scheme, errs, rates)


# ------------------------------------------- rounding-decided stop decisions
def _dd_noise(monkeypatch, seed):
    """Adds FP64-rounding-sized noise (2e-16 max|f|, absolute) to every
    divided-difference table the oracle forms."""
    orig = leja.coefficients
    rng = np.random.default_rng(seed)

    def noisy(*a, **k):
        d, fm = orig(*a, **k)
        return np.asarray(d) + 2e-16 * fm * rng.standard_normal(len(d)), fm
    monkeypatch.setattr(leja, "coefficients", noisy)


def test_adr_advection_dominated_decisions_are_rounding_decided(monkeypatch):
    # grid Peclet 2.08: the non-normal basis grows until the stop test meets
    # the divided differences' rounding floor, so rounding-level changes move
    # the substep count, while every result stays close to dense expm
    p = adr_neumann(24, alpha=0.1, beta=-5.0, rate=100.0, seed=50, amp=0.02)
    op = Operator(p)
    h = 10 * p.h_cfl
    v = h * op.rhs(p.state)
    exact = phi_dense(h * op.dense(), v, 1)
    seen = set()
    for seed in (None, 1, 2, 3):
        if seed is not None:
            _dd_noise(monkeypatch, seed)
        w, st = phi_action(op, v, 1, h, 1e-10)
        seen.add(st.substeps[0])
        assert st.converged and rel(w, exact) <= 10 * st.substeps[0] * 1e-10
        monkeypatch.undo()
    assert len(seen) >= 2


def test_adr_near_normal_decisions_are_stable(monkeypatch):
    # grid Peclet 0.1: the same perturbations leave every decision unchanged
    p = adr_neumann(96, alpha=0.1, beta=-1.0, rate=100.0, amp=0.02)
    op = Operator(p)
    h = 10 * p.h_cfl
    v = h * op.rhs(p.state)
    for l in (0, 1):
        ref = phi_action(op, v, l, h, 1e-10)[1]
        for seed in (1, 2):
            _dd_noise(monkeypatch, seed)
            st = phi_action(op, v, l, h, 1e-10)[1]
            monkeypatch.undo()
            assert st.m_star == ref.m_star and st.substeps == ref.substeps


def _mode_sum(n, modes, coef_fn, idx_i, idx_j):
    """Re(sum_k A_k c_k e^{i(2 pi (kx i + ky j)/n + theta_k)}) at points (i, j)."""
    out = np.zeros(len(idx_i))
    for kx, ky, A, th in modes:
        ph = 2 * np.pi * (kx * idx_i + ky * idx_j) / n + th
        out += (A * coef_fn(kx, ky) * np.exp(1j * ph)).real
    return out


def test_fourier_mode_closed_form_any_size():
    # the expected values of the maximum-size GPU test: for a sum of Fourier
    # modes, J acts by the symbol and phi_l(hJ) by phi_l(h sigma), point by point
    from oracle.exact import advdiff_symbol_at, phi_scalar_expm
    from workloads import fourier_modes
    n, nu = 48, 1.0
    dx = 1.0 / n
    a = nu / dx
    p = Problem("advdiff", n, n, 1, dx, dx, (nu, a, a), None, dx * dx / (4 * nu))
    op = Operator(p)
    v, modes = fourier_modes(n, 3, seed=11, kmax=12)
    jj, ii = np.divmod(np.arange(n * n), n)
    sig = lambda kx, ky: advdiff_symbol_at(2 * np.pi * kx / n, 2 * np.pi * ky / n, dx, dx, nu, a, a)
    assert np.allclose(_mode_sum(n, modes, lambda kx, ky: 1.0, ii, jj), v, atol=1e-12)
    assert np.allclose(_mode_sum(n, modes, sig, ii, jj), op.jv(v), rtol=0, atol=1e-9 * np.max(np.abs(op.jv(v))))
    h = 10 * p.h_cfl
    ref = _mode_sum(n, modes, lambda kx, ky: phi_scalar_expm(1, h * sig(kx, ky)), ii, jj)
    w, st = phi_action(op, v, 1, h, 1e-14)
    assert st.converged and rel(w, ref) <= 1e-12


def test_divided_differences_noise_regime(monkeypatch):
    """Advection-diffusion 32^2 at 100x the CFL step with four substeps (the
    learned proposal's choice for it): each substep expansion stops near
    m = 50, where the FP64 divided differences of exp at the scaled nodes
    already carry a rounding error of more than 10 % (against 100-digit
    ones), so the point counts follow the rounding of the table (Sec. 2.2,
    last paragraph) while the action stays within 10 s tol of the Fourier
    closed form."""
    import mpmath as mp
    from oracle.exact import advdiff_symbol, fourier_closed_form
    p, v = advdiff_bump()
    op = Operator(p)
    h = 100 * p.h_cfl
    lam = 8774.344002821865
    c, gamma = leja.interval(lam, 1.25)
    tau = h / 4
    xi = leja.xi_table(101)
    d64, _ = leja.coefficients(0, 1.0, tau, c, gamma, 56)
    mp.mp.dps = 100
    xs = [mp.mpf(x) for x in xi[:56]]
    d = [mp.e ** (mp.mpf(tau) * (mp.mpf(c) + mp.mpf(gamma) * x)) for x in xs]
    for k in range(1, 56):
        for j in range(55, k - 1, -1):
            d[j] = (d[j] - d[j - 1]) / (xs[j] - xs[j - k])
    relerr = [abs(d64[m] - float(d[m])) / abs(float(d[m])) for m in range(56)]
    assert max(relerr[:30]) < 1e-9 and relerr[50] > 0.1
    sig = advdiff_symbol(p.nx, p.ny, p.dx, p.dy, *p.coef)
    exact = fourier_closed_form(sig, v, 3, h)
    # one-ulp changes of the node values (two exp implementations differ by
    # that much) move the counts
    orig = leja.phi
    counts = set()
    for seed in (None, 1, 2, 3):
        if seed is not None:
            rng = np.random.default_rng(seed)
            monkeypatch.setattr(leja, "phi", lambda l, z: orig(l, z) * (1.0 + 2.0 ** -52 * rng.integers(-1, 2)))
        w, st = phi_action(op, v, 3, h, 1e-10, Options(bound=lam, substeps=4, max_substeps=4))
        monkeypatch.undo()
        counts.add(st.m_star[0])
        assert st.converged and rel(w, exact) <= 10 * 4 * 1e-10
    assert len(counts) >= 2


def test_dd_floor_of_long_expansion(monkeypatch):
    """Allen-Cahn 64^2 (eps 1e-2) at 100x the CFL step, phi_1, 88 Newton
    terms: the FP64 table's entries near the stop carry ~1e-2..1e-1 rounding
    error, which moves the action by more than 1e-10 relative to the same
    expansion with exact coefficients; at 10x the CFL step the floor is far
    below tol.  The exact table itself matches the FP64 one where the latter
    is accurate (low orders)."""
    from dd_floor import dd_floor, exact_coefficients
    p = allen_cahn_noise(64, eps=1e-2, seed=3)
    op = Operator(p)
    lam = 86.93866065109043
    c, gamma = leja.interval(lam, 1.25)
    h = 100 * p.h_cfl
    d64, f64 = leja.coefficients(1, 1.0, h, c, gamma, 101)
    dex, fex = exact_coefficients(1, 1.0, h, c, gamma, 101)
    assert np.max(np.abs(d64[:30] - dex[:30]) / np.abs(dex[:30])) < 1e-12 and abs(f64 - fex) <= 1e-15 * fex
    assert abs(d64[83] - dex[83]) > 0.05 * abs(dex[83])
    v = h * op.rhs(p.state)
    run = lambda: phi_action(op, v, 1, h, 1e-10, Options(bound=lam))[0]
    assert dd_floor(monkeypatch, run, rel) > 1e-10
    h10 = 10 * p.h_cfl
    v10 = h10 * op.rhs(p.state)
    run10 = lambda: phi_action(op, v10, 1, h10, 1e-10, Options(bound=lam))[0]
    assert dd_floor(monkeypatch, run10, rel) < 1e-13


def test_batch_rejection_regime_is_rounding_decided():
    """Instance 46 of the 256-instance ensemble (128^2, eps 1.5e-4, h 10x
    CFL): the reaction eigenvalue +1 lies outside the interval, the Newton
    basis grows, and whether the attempts at s = 2, 4 pass the hump test is
    decided by the rounding of the divided differences -- one-ulp changes of
    the node values move the substep count between 4 and 8, while each run
    converges."""
    from oracle.power import power_iteration
    from workloads import batch_instances
    p = batch_instances()[46]
    op = Operator(p)
    h = 10 * p.h_cfl
    v = h * op.rhs(p.state)
    lam = power_iteration(op.jv, p.n, 20)
    orig = leja.phi
    seen = set()
    try:
        for seed in (None, 1, 3):
            if seed is not None:
                rng = np.random.default_rng(seed)
                leja.phi = lambda l, z: orig(l, z) * (1.0 + 2.0 ** -52 * rng.integers(-1, 2))
            _, so = phi_vertical(op, v, [1, 2, 3], [1.0] * 3, h, 1e-10, Options(bound=lam))
            leja.phi = orig
            assert so.converged
            seen.add(max(so.substeps))
    finally:
        leja.phi = orig
    assert seen == {4, 8}
