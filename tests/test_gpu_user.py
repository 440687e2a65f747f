"""GPU tests of the user-operator path (lj_user_*, lj_jv): operators given as
callbacks, with the Newton recurrence, stop decisions, power iteration,
substepping and schemes in the library's kernels.  Checked against the CPU
oracle on the same inputs: a built-in family seen through its own callbacks
(bound forced equal: 1e-10 and identical m*), finite-difference products
(bar set by the products' own ~1e-8 error), and the 1-D semilinear problem of
Sec. 3 written as torch callbacks, integrated to t = 1 and compared with the
oracle step by step and with the paper's exact solution."""

import numpy as np
import pytest

from gpu_util import rel, rel2, say
from oracle.fdjac import FDOperator
from oracle.integrators import step as oracle_step
from oracle.leja import Options, phi_action, phi_vertical
from oracle.operators import Operator
from oracle.power import power_iteration
from oracle.semilinear import Semilinear
from workloads import (adr_neumann, advdiff_bump, allen_cahn_noise, brusselator_perturbed, burgers_sines,
                       diag_problem, gray_scott_spots)

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2211_08948_amd as lj
    ctx = lj.Context(0)
    yield lj, torch, ctx
    ctx.close()


def _dev(torch, x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda:0").contiguous()


FAMILIES = {
    "diag": lambda: diag_problem(1000, -300.0, seed=3),
    "advdiff": lambda: advdiff_bump()[0],
    "allencahn": lambda: allen_cahn_noise(37, eps=1e-1, seed=7),
    "brusselator": lambda: brusselator_perturbed(48, D=2e-2, seed=3),
    "burgers": lambda: burgers_sines(64, nu=3e-2, seed=5),
    "grayscott": lambda: gray_scott_spots(40, a1=2e-2, a2=1e-2, amp=0.02),
    "adr": lambda: adr_neumann(37, alpha=0.3, beta=-1.0, rate=100.0, amp=0.02),
}


@pytest.mark.parametrize("name", list(FAMILIES))
def test_family_jv_parity(env, name):
    lj, torch, ctx = env
    prob = FAMILIES[name]()
    say("lj_jv", name)
    J = lj.operator_from(prob, "cuda:0")
    x = np.random.default_rng(4).uniform(-1, 1, prob.n)
    y = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    lj.lj_jv(ctx, J, _dev(torch, x), y)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), Operator(prob).jv(x)) <= 1e-14


def _ac():
    prob = allen_cahn_noise(96, eps=2e-2, seed=2)
    op = Operator(prob)
    h = 10 * prob.h_cfl
    return prob, op, h, h * op.rhs(prob.state)


@pytest.mark.parametrize("l", [0, 1, 3])
def test_user_action_parity(env, l):
    lj, torch, ctx = env
    prob, op, h, v = _ac()
    w_orc, st_orc = phi_action(op, v, l, h, TOL)
    say("user action", l, st_orc.m_star)
    J = lj.operator_from(prob, "cuda:0")
    U = lj.family_user_operator(ctx, J)
    w = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    rc, st = lj.lj_user_phi_action(ctx, U, _dev(torch, v), w, l, h, TOL, lj.lj_default_options(bound=st_orc.bound))
    assert rc == 0 and st["m_star"] == st_orc.m_star and st["substeps"] == st_orc.substeps
    assert st["iters_total"] == st_orc.iters_total
    assert st["c"] == st_orc.c and st["gamma"] == st_orc.gamma
    assert rel(w.cpu().numpy(), w_orc) <= TOL


def test_user_own_power_iteration_vertical_and_forced_substeps(env):
    lj, torch, ctx = env
    prob, op, h, v = _ac()
    J = lj.operator_from(prob, "cuda:0")
    U = lj.family_user_operator(ctx, J)
    vd = _dev(torch, v)
    # own power iteration on both sides, vertical EPIRK4s3 coefficients
    ls, As = [1, 1, 1], [1 / 8, 1 / 9, 1.0]
    wo, so = phi_vertical(op, v, ls, As, h, TOL)
    ws = [torch.empty_like(vd) for _ in ls]
    rc, st = lj.lj_user_phi_vertical(ctx, U, vd, ls, As, h, TOL, ws)
    say("user vertical", st["m_star"], so.m_star, st["bound"], so.bound)
    assert rc == 0 and st["power_iters"] == 20 and abs(st["bound"] - so.bound) <= 1e-12 * so.bound
    lam = so.bound
    ws2 = [torch.empty_like(vd) for _ in ls]
    rc, st = lj.lj_user_phi_vertical(ctx, U, vd, ls, As, h, TOL, ws2, lj.lj_default_options(bound=lam))
    assert st["m_star"] == so.m_star
    for k in range(3):
        assert rel(ws2[k].cpu().numpy(), wo[k]) <= TOL
    # substeps forced from the start (Sec. 2.2 substepping on every path)
    for l in (1, 3):
        w_orc, st_orc = phi_action(op, v, l, h, TOL, Options(bound=lam, substeps=4))
        w = torch.empty_like(vd)
        rc, st = lj.lj_user_phi_action(ctx, U, vd, w, l, h, TOL, lj.lj_default_options(bound=lam, substeps=4))
        say("user substeps", l, st["m_star"], st_orc.m_star)
        assert rc == 0 and st["substeps"] == st_orc.substeps == [4] and st["m_star"] == st_orc.m_star
        assert rel(w.cpu().numpy(), w_orc) <= TOL


@pytest.mark.parametrize("scheme", ["EXPRB43", "EPIRK4S3"])
def test_user_step_parity(env, scheme):
    lj, torch, ctx = env
    prob, op, h, _ = _ac()
    lam = power_iteration(op.jv, prob.n, 20)
    u_orc, e_orc, log = oracle_step(op, scheme, h, TOL, Options(bound=lam))
    J = lj.operator_from(prob, "cuda:0")
    U = lj.family_user_operator(ctx, J)
    u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    err = torch.empty_like(u_out)
    rc, sts = lj.lj_user_step(ctx, scheme, U, h, TOL, u_out, err, lj.lj_default_options(bound=lam))
    say("user step", scheme, [s["m_star"][:3] for s in sts])
    assert rc == 0 and [s["m_star"][:len(b.m_star)] for s, b in zip(sts, log)] == [b.m_star for b in log]
    assert rel(u_out.cpu().numpy(), u_orc) <= TOL
    assert np.linalg.norm(err.cpu().numpy() - e_orc) <= 1e-8 * np.linalg.norm(e_orc) + 1e-12 * np.linalg.norm(u_orc)


@pytest.mark.parametrize("l", [0, 1])
def test_user_finite_difference_action(env, l):
    """rhs only: the library forms J v by forward differences.  The two sides'
    products differ by their own rounding, ~2^-52 ||f|| / eps ~ 1e-8 relative
    per product, which the expansion carries into the result (the oracle's FD
    result is 5e-6 from its analytic one for l = 0): results within 2e-5 of
    both oracle results, point counts within 2."""
    lj, torch, ctx = env
    prob, op, h, v = _ac()
    lam = power_iteration(op.jv, prob.n, 20)
    w_an, st_an = phi_action(op, v, l, h, TOL, Options(bound=lam))
    w_fd, st_fd = phi_action(FDOperator(op), v, l, h, TOL, Options(bound=lam))
    J = lj.operator_from(prob, "cuda:0")
    U = lj.family_user_operator(ctx, J, finite_difference=True)
    w = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    rc, st = lj.lj_user_phi_action(ctx, U, _dev(torch, v), w, l, h, TOL, lj.lj_default_options(bound=lam))
    say("user fd", l, st["m_star"], st_fd.m_star, st_an.m_star)
    assert rc == 0 and st["converged"]
    assert abs(st["m_star"][0] - st_fd.m_star[0]) <= 2
    wg = w.cpu().numpy()
    assert rel2(wg, w_fd) <= 2e-5 and rel2(wg, w_an) <= 2e-5
    # the finite-difference power iteration lands on the analytic bound
    rc, st2 = lj.lj_user_phi_action(ctx, U, _dev(torch, v), w, l, h, TOL)
    assert abs(st2["bound"] - lam) <= 1e-6 * lam


def test_user_zero_vector_and_errors(env):
    lj, torch, ctx = env
    prob, op, h, v = _ac()
    J = lj.operator_from(prob, "cuda:0")
    U = lj.family_user_operator(ctx, J)
    z = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")
    w = torch.full_like(z, 7.0)
    rc, st = lj.lj_user_phi_action(ctx, U, z, w, 1, h, TOL, lj.lj_default_options(bound=100.0))
    assert rc == 0 and st["m_star"] == [0] and torch.count_nonzero(w).item() == 0
    # a callback that raises: the call fails and the exception is chained
    def bad(u, x, out):
        raise ValueError("planted failure in a user callback")
    Ub = lj.UserOperator(prob.n, J.state, jv=bad)
    with pytest.raises(lj.LejaError) as ei:
        lj.lj_user_phi_action(ctx, Ub, _dev(torch, v), w, 1, h, TOL, lj.lj_default_options(bound=100.0))
    assert isinstance(ei.value.__cause__, ValueError)
    # a callback may not re-enter the library's workspace-using entry points
    def reenter(u, x, out):
        lj.lj_phi_action(ctx, J, x, out, 1, h, TOL, lj.lj_default_options(bound=100.0))
    Ur = lj.UserOperator(prob.n, J.state, jv=reenter)
    with pytest.raises(lj.LejaError) as ei:
        lj.lj_user_phi_action(ctx, Ur, _dev(torch, v), w, 1, h, TOL, lj.lj_default_options(bound=100.0))
    assert isinstance(ei.value.__cause__, lj.LejaError) and "callbacks" in str(ei.value.__cause__)
    # the stage driver needs rhs; the proposal needs a built-in family
    Uj = lj.UserOperator(prob.n, J.state, jv=lambda u, x, out: lj.lj_jv(ctx, J, x, out))
    with pytest.raises(lj.LejaError):
        lj.lj_user_step(ctx, "EXPRB2", Uj, h, TOL, w)
    with pytest.raises(lj.LejaError):
        lj.lj_user_phi_action(ctx, U, _dev(torch, v), w, 1, h, TOL, lj.lj_default_options(use_proposal=1))
    # the context still works afterwards
    lam = power_iteration(op.jv, prob.n, 20)
    rc, st = lj.lj_user_phi_action(ctx, U, _dev(torch, v), w, 1, h, TOL, lj.lj_default_options(bound=lam))
    assert rc == 0 and st["m_star"] == phi_action(op, v, 1, h, TOL, Options(bound=lam))[1].m_star


class TorchSemilinear:
    """The semilinear problem of Sec. 3 as torch callbacks (user code: the
    grid, Simpson weights and forcing written independently of the oracle)."""

    def __init__(self, torch, N):
        self.t = torch
        self.N = N
        self.dx = 1.0 / (N + 1)
        i = torch.arange(1, N + 1, dtype=torch.float64, device="cuda:0")
        self.x = i * self.dx
        self.w = (2.0 + 2.0 * torch.remainder(i, 2.0)) * (self.dx / 3.0)  # 4, 2, 4, ..., 4
        self.g = self.x * (1.0 - self.x) + 11.0 / 6.0

    def d2(self, u):
        p = self.t.nn.functional.pad(u, (1, 1))
        return (p[:-2] - 2.0 * p[1:-1] + p[2:]) / (self.dx * self.dx)

    def rhs(self, X, out):
        N = self.N
        u = X[:N]
        out[:N] = self.d2(u) + self.t.dot(self.w, u) + self.t.exp(X[N]) * self.g
        out[N] = 1.0

    def jv(self, U, X, out):
        N = self.N
        v = X[:N]
        out[:N] = self.d2(v) + self.t.dot(self.w, v) + self.t.exp(U[N]) * self.g * X[N]
        out[N] = 0.0


@pytest.mark.parametrize("scheme", ["EXPRB43", "EPIRK4S3", "EPIRK4S3_LEKRY", "EPIRK4S3A"])
def test_semilinear_end_to_end(env, scheme):
    """Eight steps of h = 1/8 to t = 1 from the exact initial state; each step
    linearised at the GPU's own state with the oracle's bound at the oracle's
    state (the states agree to rounding).  Per-step point counts equal, final
    states within 1e-9, and both within the scheme's own error of the exact
    solution x(1-x)e (the oracle's error, pinned on the CPU by its order)."""
    lj, torch, ctx = env
    N = 31
    ts = TorchSemilinear(torch, N)
    Uo = Semilinear(N).exact(0.0)
    Ug = _dev(torch, Uo)
    nsteps = 8
    h = 1.0 / nsteps
    for k in range(nsteps):
        op = Semilinear(N, Uo)
        lam = power_iteration(op.jv, op.n, 20)
        Uo, _, log = oracle_step(op, scheme, h, TOL, Options(bound=lam))
        U = lj.UserOperator(N + 1, Ug, rhs=ts.rhs, jv=ts.jv)
        out = torch.empty_like(Ug)
        rc, sts = lj.lj_user_step(ctx, scheme, U, h, TOL, out, None, lj.lj_default_options(bound=lam))
        assert rc == 0
        assert [s["m_star"][:len(b.m_star)] for s, b in zip(sts, log)] == [b.m_star for b in log], k
        Ug = out
    ug = Ug.cpu().numpy()
    exact = Semilinear(N).exact(1.0)
    e_orc = rel2(Uo, exact)
    say("semilinear", scheme, "gpu vs oracle", rel2(ug, Uo), "oracle vs exact", e_orc, "gpu vs exact", rel2(ug, exact))
    assert rel2(ug, Uo) <= 1e-9
    assert rel2(ug, exact) <= 1.01 * e_orc + 1e-9
    assert e_orc < 1e-5


def test_semilinear_variable_steps(env):
    """Variable step sizes (Sec. 2.3) on the semilinear problem through the
    callbacks: the same accepted and rejected attempts, step sizes and
    product counts as the oracle's controller, the same u(1), and the exact
    solution to within the accumulated step tolerances."""
    from oracle import adaptive as A
    lj, torch, ctx = env
    N = 31
    u0 = Semilinear(N).exact(0.0)
    orc = A.integrate(None, u0, 1.0, 0.05, 1e-6, "EPIRK4S3", leja_tol=TOL, make_op=lambda u: Semilinear(N, u))
    ts = TorchSemilinear(torch, N)
    U = lj.UserOperator(N + 1, _dev(torch, u0), rhs=ts.rhs, jv=ts.jv)
    out = torch.empty_like(U.state)
    rc, st, recs = lj.lj_user_integrate(ctx, "EPIRK4S3", U, 1.0, 0.05, 1e-6, TOL, out)
    say("semilinear adaptive", st, orc.accepted, orc.rejected, orc.products)
    assert rc == 0 and st["t"] == 1.0
    assert (st["accepted"], st["rejected"], st["products"]) == (orc.accepted, orc.rejected, orc.products)
    for r, a in zip(recs, orc.attempts):
        assert r["accepted"] == a.accepted and r["products"] == a.cost
        # sizes follow (tol / e)^{1/4}; e is the norm of the difference of two
        # close solutions, whose rounding leaves ~1e-5 of it different
        assert r["dt"] == pytest.approx(a.dt, rel=1e-4)
    u = out.cpu().numpy()
    exact = Semilinear(N).exact(1.0)
    assert rel(u, orc.u) <= 1e-9
    assert rel2(u, exact) <= 1e-6
