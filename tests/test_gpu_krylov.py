"""GPU tests of the Krylov evaluation of phi combinations (lj_phi_combination,
lj_user_phi_combination) and of the LeKry step: against the CPU oracle on the
same inputs (identical substep, rejection and product counts -- the cases
keep every accept/reject ratio at least 15 % away from 1 -- and results
within 1e-11), against dense Pade expm of the augmented matrix, and LeKry
against EPIRK4s3."""
import numpy as np
import pytest

from gpu_util import rel, rel2, say
from oracle.exact import phi_dense
from oracle.integrators import step as oracle_step
from oracle.krylov import KrylovOptions, phi_combination
from oracle.leja import Options
from oracle.operators import Operator
from oracle.power import power_iteration
from workloads import advdiff_bump, allen_cahn_noise, brusselator_perturbed

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


CASES = {
    "allencahn": lambda: allen_cahn_noise(96, eps=2e-2, seed=2),
    "advdiff": lambda: advdiff_bump()[0],
    "brusselator": lambda: brusselator_perturbed(48, D=2e-2, seed=3),
}


def _bs(prob):
    rng = np.random.default_rng(1)
    return [rng.uniform(-1, 1, prob.n), rng.uniform(-1, 1, prob.n), None, rng.uniform(-1, 1, prob.n)]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("window", [2, 8, 0])
@pytest.mark.parametrize("mult,m", [(10, 30), (30, 10)])
def test_combination_parity(env, name, window, mult, m):
    lj, torch, ctx = env
    prob = CASES[name]()
    op = Operator(prob)
    h = mult * prob.h_cfl
    bs = _bs(prob)
    w_orc, st_orc = phi_combination(op.jv, bs, h, TOL, KrylovOptions(m=m, window=window))
    J = lj.operator_from(prob, "cuda:0")
    w = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    rc, st = lj.lj_phi_combination(ctx, J, [None if b is None else _dev(torch, b) for b in bs], h, TOL, w,
                                   lj.lj_default_krylov_options(krylov_dim=m, window=window))
    say("krylov", name, window, mult, m, st["substeps"], st["rejections"], st["iters_total"], "oracle",
        st_orc.substeps, st_orc.rejections, st_orc.products)
    assert rc == 0 and st["converged"]
    assert st["substeps"] == [st_orc.substeps] and st["rejections"] == st_orc.rejections
    assert st["iters_total"] == st_orc.products
    assert rel(w.cpu().numpy(), w_orc) <= 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_persistent_basis_matches_passes(env, name, monkeypatch):
    """Windows of 1 or 2 vectors build the basis in one persistent launch; the
    hook LJ_KRYLOV_PASSES=1 forces the four-launches-per-column kernels.  The
    two differ only in the order of the dot products' partial sums."""
    lj, torch, ctx = env
    prob = CASES[name]()
    h = 30 * prob.h_cfl
    bs = [None if b is None else _dev(torch, b) for b in _bs(prob)]
    J = lj.operator_from(prob, "cuda:0")
    monkeypatch.setenv("LJ_KRYLOV_PASSES", "1")
    ctx_p = lj.Context(0)
    monkeypatch.delenv("LJ_KRYLOV_PASSES")
    for window in (1, 2):
        ko = lj.lj_default_krylov_options(krylov_dim=30, window=window)
        w1 = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
        w2 = torch.empty_like(w1)
        rc1, st1 = lj.lj_phi_combination(ctx, J, bs, h, TOL, w1, ko)
        rc2, st2 = lj.lj_phi_combination(ctx_p, J, bs, h, TOL, w2, ko)
        say("persistent vs passes", name, window, st1["substeps"], st2["substeps"], st1["iters_total"])
        assert rc1 == rc2 == 0
        assert st1["substeps"] == st2["substeps"] and st1["rejections"] == st2["rejections"]
        assert st1["iters_total"] == st2["iters_total"]
        assert rel(w1.cpu().numpy(), w2.cpu().numpy()) <= 1e-13
    ctx_p.close()


@pytest.mark.parametrize("passes", [False, True])
def test_exact_breakdown(env, passes, monkeypatch):
    """A constant on the periodic advection-diffusion grid: J c = 0 exactly, so
    with b_0 = c (and b_1 = 0) A~ maps the start vector to 0 and the basis
    ends at the breakdown after one vector: the projection is exact, one
    substep, w = c.  With b_1 = c the space is invariant after two vectors
    only up to rounding (A~ [c; 1] = [c; 0], A~ [c; 0] = 0): no breakdown in
    floating point, the full basis is built on the rounding residue, and the
    result is still c + h c."""
    lj, torch, ctx0 = env
    if passes:
        monkeypatch.setenv("LJ_KRYLOV_PASSES", "1")
    ctx = lj.Context(0)
    monkeypatch.delenv("LJ_KRYLOV_PASSES", raising=False)
    prob = CASES["advdiff"]()
    op = Operator(prob)
    c = np.full(prob.n, 0.75)
    J = lj.operator_from(prob, "cuda:0")
    w = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    h = 30 * prob.h_cfl
    for bs, expect, prods in (([c], c, 1), ([c, 0 * c], c, 1), ([c, c], c + h * c, 30)):
        w_orc, st_orc = phi_combination(op.jv, bs, h, TOL, KrylovOptions())
        assert st_orc.products == prods and st_orc.substeps == 1
        rc, st = lj.lj_phi_combination(ctx, J, [_dev(torch, b) for b in bs], h, TOL, w)
        say("breakdown", "passes" if passes else "persistent", len(bs), st["iters_total"], st["substeps"])
        assert rc == 0 and st["iters_total"] == prods and st["substeps"] == [1] and st["rejections"] == 0
        assert rel(w.cpu().numpy(), expect) <= 1e-14 and rel(w_orc, expect) <= 1e-14
    ctx.close()


def test_combination_matches_dense_pade(env):
    lj, torch, ctx = env
    prob = allen_cahn_noise(16, eps=1e-2, seed=8)
    prob.state = prob.state * 8
    op = Operator(prob)
    h = 10 * prob.h_cfl
    rng = np.random.default_rng(5)
    bs = [rng.uniform(-1, 1, prob.n), None, rng.uniform(-1, 1, prob.n), None, rng.uniform(-1, 1, prob.n)]
    ref = sum(phi_dense(h * op.dense(), b, j) * h ** j for j, b in enumerate(bs) if b is not None)
    J = lj.operator_from(prob, "cuda:0")
    w = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    for tol in (1e-10, 1e-13):
        rc, st = lj.lj_phi_combination(ctx, J, [None if b is None else _dev(torch, b) for b in bs], h, tol, w)
        assert rc == 0 and rel2(w.cpu().numpy(), ref) <= 10 * tol + 1e-14


def test_combination_edge_cases(env):
    lj, torch, ctx = env
    prob = CASES["allencahn"]()
    J = lj.operator_from(prob, "cuda:0")
    b0 = _dev(torch, np.random.default_rng(2).uniform(-1, 1, prob.n))
    w = torch.empty_like(b0)
    # h = 0: phi_0(0) b_0 = b_0 and every other term carries h^j = 0
    rc, st = lj.lj_phi_combination(ctx, J, [b0, b0], 0.0, TOL, w)
    assert rc == 0 and torch.equal(w, b0)
    # all terms zero
    rc, st = lj.lj_phi_combination(ctx, J, [None], 0.1, TOL, w)
    assert rc == 0 and torch.count_nonzero(w).item() == 0
    for bad in (dict(bs=[b0] * 6), dict(h=-1.0), dict(tol=0.0)):
        kw = dict(bs=[b0, b0], h=0.1, tol=TOL)
        kw.update(bad)
        with pytest.raises(lj.LejaError):
            lj.lj_phi_combination(ctx, J, kw["bs"], kw["h"], kw["tol"], w)
    with pytest.raises(lj.LejaError):
        lj.lj_phi_combination(ctx, J, [b0, b0], 0.1, TOL, b0)  # w aliases b_0
    with pytest.raises(lj.LejaError):
        lj.lj_phi_combination(ctx, J, [b0], 0.1, TOL, w, lj.lj_default_krylov_options(krylov_dim=65))


def test_user_combination_parity(env):
    lj, torch, ctx = env
    prob = CASES["advdiff"]()
    op = Operator(prob)
    h = 30 * prob.h_cfl
    bs = _bs(prob)
    w_orc, st_orc = phi_combination(op.jv, bs, h, TOL, KrylovOptions(m=10))
    J = lj.operator_from(prob, "cuda:0")
    J.state = torch.zeros(prob.n, dtype=torch.float64, device="cuda:0")  # the linear operator needs no state
    U = lj.UserOperator(prob.n, J.state, jv=lambda u, x, out: lj.lj_jv(ctx, J, x, out))
    w = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    rc, st = lj.lj_user_phi_combination(ctx, U, [None if b is None else _dev(torch, b) for b in bs], h, TOL, w,
                                        lj.lj_default_krylov_options(krylov_dim=10))
    assert rc == 0 and st["substeps"] == [st_orc.substeps] and st["iters_total"] == st_orc.products
    assert rel(w.cpu().numpy(), w_orc) <= 1e-11


@pytest.mark.parametrize("base", ["EPIRK4S3", "EPIRK4S3A"])
def test_lekry_step_parity(env, base):
    lj, torch, ctx = env
    prob = allen_cahn_noise(96, eps=2e-2, seed=2)
    op = Operator(prob)
    h = 10 * prob.h_cfl
    lam = power_iteration(op.jv, prob.n, 20)
    u_orc, e_orc, log = oracle_step(op, base + "_LEKRY", h, TOL, Options(bound=lam))
    J = lj.operator_from(prob, "cuda:0")
    u_out = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    err = torch.empty_like(u_out)
    rc, sts = lj.lj_step(ctx, base + "_LEKRY", J, h, TOL, u_out, err, lj.lj_default_options(bound=lam))
    say("lekry", [s["m_star"][:2] for s in sts], [b.m_star for b in log])
    assert rc == 0 and len(sts) == 3
    assert sts[0]["m_star"][:2] == log[0].m_star and sts[2]["m_star"][:1] == log[2].m_star
    assert sts[1]["substeps"][0] == log[1].substeps[0] and sts[1]["iters_total"] == log[1].iters_total
    assert rel(u_out.cpu().numpy(), u_orc) <= TOL
    assert np.linalg.norm(err.cpu().numpy() - e_orc) <= 1e-8 * np.linalg.norm(e_orc) + 1e-12 * np.linalg.norm(u_orc)
    # the same scheme as the all-Leja form, its third stage evaluated by Krylov
    u4 = torch.empty_like(u_out)
    rc, _ = lj.lj_step(ctx, base, J, h, TOL, u4, None, lj.lj_default_options(bound=lam))
    assert rel(u_out.cpu().numpy(), u4.cpu().numpy()) <= 1e-9
