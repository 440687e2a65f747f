"""Deferred synchronisation (lj_defer_begin / lj_defer_end) through the C
ABI: a deferred sequence of steps and actions gives the same results and
statistics as the same calls made one by one; a deferred call whose
expansion is rejected is redone, with the deferred calls after it, at
lj_defer_end; calls that cannot be deferred are argument errors."""
import numpy as np
import pytest

from gpu_util import rel, say
from workloads import allen_cahn_noise

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2211_08948_amd as lj
    ctx = lj.Context(0)
    yield lj, torch, ctx
    ctx.close()


def _setup(lj, torch, ctx, n=96, eps=2e-2, mult=10.0):
    prob = allen_cahn_noise(n, eps=eps, seed=2)
    J = lj.operator_from(prob, "cuda:0")
    h = mult * prob.h_cfl
    f = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
    lj.lj_rhs(ctx, J, J.state, f)
    v = (h * f).contiguous()
    return prob, J, h, v


def _bench_like_calls(lj, torch, ctx, J, h, v, opt=None):
    """EXPRB2 step, EPIRK4s3 step, phi_2 on the EPIRK4s3 bound -- one by one."""
    u2 = torch.empty_like(v)
    u4 = torch.empty_like(v)
    err = torch.empty_like(v)
    w = torch.empty_like(v)
    _, s2 = lj.lj_step(ctx, "EXPRB2", J, h, TOL, u2, None, opt)
    _, s4 = lj.lj_step(ctx, "EPIRK4S3", J, h, TOL, u4, err, opt)
    o = lj.lj_default_options(bound=s4[0]["bound"])
    if opt is not None:
        o.max_points = opt.max_points
    _, s1 = lj.lj_phi_action(ctx, J, v, w, 2, h, TOL, o)
    torch.cuda.synchronize()
    return (u2, u4, err, w), (s2, s4, s1)


def test_deferred_sequence_matches_one_by_one(env):
    lj, torch, ctx = env
    prob, J, h, v = _setup(lj, torch, ctx)
    ref, (r2, r4, r1) = _bench_like_calls(lj, torch, ctx, J, h, v)
    u2, u4, err, w = (torch.empty_like(v) for _ in range(4))
    with lj.Deferred(ctx) as d:
        d.step("EXPRB2", J, h, TOL, u2, None)
        d.step("EPIRK4S3", J, h, TOL, u4, err)
        d.phi_action(J, v, w, 2, h, TOL, lj.lj_default_options(bound_device=lj.lj_bound_device(ctx)))
    (rc2, s2), (rc4, s4), (rc1, s1) = d.results
    say("deferred", s2[0]["m_star"], s4[0]["m_star"], s1["m_star"])
    assert d.rc == 0
    assert s2 == r2 and s4 == r4
    for key in ("m_star", "iters_total", "bound", "substeps"):
        assert s1[key] == r1[key], key
    for a, b in zip((u2, u4, err, w), ref):
        assert torch.equal(a, b)


def test_deferred_rejection_is_redone_in_order(env):
    """max_points 12 at 10x CFL: the expansions are rejected in the deferred
    pass, so lj_defer_end redoes the first call and every later one with
    substeps -- including a step whose state is the first step's output."""
    lj, torch, ctx = env
    prob, J, h, v = _setup(lj, torch, ctx)
    opt = lj.lj_default_options(max_points=12)
    u1 = torch.empty_like(v)
    _, r1 = lj.lj_step(ctx, "EXPRB2", J, h, TOL, u1, None, opt)
    J2 = lj.Operator(J.kind, J.nx, J.ny, J.ncomp, J.dx, J.dy, J.coef, u1)
    u2 = torch.empty_like(v)
    _, r2 = lj.lj_step(ctx, "EXPRB2", J2, h, TOL, u2, None, opt)
    torch.cuda.synchronize()
    assert r1[0]["rejections"] >= 1
    d1 = torch.full_like(v, float("nan"))
    d2 = torch.full_like(v, float("nan"))
    K2 = lj.Operator(J.kind, J.nx, J.ny, J.ncomp, J.dx, J.dy, J.coef, d1)
    with lj.Deferred(ctx) as d:
        d.step("EXPRB2", J, h, TOL, d1, None, opt)
        d.step("EXPRB2", K2, h, TOL, d2, None, opt)
    (_, s1), (_, s2) = d.results
    say("redo", s1[0]["substeps"], s1[0]["rejections"], s2[0]["substeps"])
    assert d.rc == 0 and s1 == r1 and s2 == r2
    assert rel(d1.cpu().numpy(), u1.cpu().numpy()) == 0.0 and rel(d2.cpu().numpy(), u2.cpu().numpy()) == 0.0


def test_deferral_argument_errors(env):
    lj, torch, ctx = env
    prob, J, h, v = _setup(lj, torch, ctx, n=32)
    w = torch.empty_like(v)
    with pytest.raises(lj.LejaError):  # no deferral open
        ctx._check(ctx._lib.lj_defer_end(ctx.handle, None), False)
    with lj.Deferred(ctx) as d:
        with pytest.raises(lj.LejaError):  # nested
            ctx._check(ctx._lib.lj_defer_begin(ctx.handle), False)
        with pytest.raises(lj.LejaError, match="deferred"):
            d.phi_action(J, v, w, 1, h, TOL, lj.lj_default_options(substeps=2))
        d.phi_action(J, v, w, 1, h, TOL)
    assert d.rc == 0 and d.results[0][1]["m_star"][0] > 0
    # the context works normally afterwards
    rc, st = lj.lj_phi_action(ctx, J, v, w, 1, h, TOL)
    assert rc == 0 and st["m_star"] == d.results[0][1]["m_star"]
    assert np.isfinite(w.cpu().numpy()).all()
