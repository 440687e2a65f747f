"""GPU tests of the batching form (lj_batch_*): many independent Allen-Cahn
instances, phi_1, phi_2, phi_3 of h_i f(u_i) on one Newton basis per
instance, all in one persistent graph-captured launch.  Checked against the
CPU oracle on small batches (bound forced equal, or each side's own power
iteration), against the plain GPU path on the full 256-instance ensemble, and
for schedule independence, graph replays, rejection fallback and argument
errors."""
import os

import numpy as np
import pytest

from gpu_util import rel, rel2, say
from oracle.leja import Options, phi_vertical
from oracle.operators import Operator
from oracle.power import power_iteration
from workloads import adr_neumann, allen_cahn_noise, batch_instances

pytestmark = pytest.mark.gpu
TOL = 1e-10
LS = [1, 2, 3]
AS = [1.0, 1.0, 1.0]


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2211_08948_amd as lj
    ctx = lj.Context(0)
    yield lj, torch, ctx
    ctx.close()


def small_set():
    """Six instances of uneven (and odd) sizes; diffusion-dominated so the
    spectrum stays inside the scaled interval."""
    spec = [(24, 0.05), (37, 0.1), (48, 0.02), (31, 0.05), (64, 0.03), (20, 0.2)]
    probs = [allen_cahn_noise(n, eps, seed=4000 + i) for i, (n, eps) in enumerate(spec)]
    hs = [10.0 * p.h_cfl for p in probs]
    vs = [h * Operator(p).rhs(p.state) for p, h in zip(probs, hs)]
    return probs, hs, vs


def make_batch(lj, torch, ctx, probs, hs, vs, bounds=None, opt=None, K=3):
    ops = [lj.operator_from(p, "cuda:0") for p in probs]
    vd = [torch.as_tensor(v, dtype=torch.float64, device="cuda:0").contiguous() for v in vs]
    ws = [[torch.empty_like(v) for _ in range(K)] for v in vd]
    b = lj.Batch(ctx, ops, vd, hs, LS[:K], AS[:K], TOL, ws, bounds=bounds, opt=opt)
    return b, ws, (ops, vd)


def test_batch_matches_oracle_with_oracle_bound(env):
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    bounds = [power_iteration(Operator(p).jv, p.n) for p in probs]
    b, ws, _ = make_batch(lj, torch, ctx, probs, hs, vs, bounds=bounds)
    b.run()
    rc, sts = b.stats()
    assert rc == 0
    for i, (p, h, v) in enumerate(zip(probs, hs, vs)):
        wo, so = phi_vertical(Operator(p), v, LS, AS, h, TOL, Options(bound=bounds[i]))
        st = sts[i]
        say("batch vs oracle", i, p.nx, st["m_star"], so.m_star)
        assert st["m_star"] == so.m_star and st["substeps"] == so.substeps
        assert st["bound"] == bounds[i] and st["c"] == so.c and st["gamma"] == so.gamma
        assert st["power_iters"] == 0 and st["rejections"] == 0
        for k in range(3):
            assert rel(ws[i][k].cpu().numpy(), wo[k]) <= TOL
    b.close()


def test_batch_adr_neumann_matches_oracle(env):
    # a batch of advection-diffusion-reaction instances (Neumann boundaries,
    # Sec. 3 initial state plus noise, grid Peclet number <= 0.42), each side
    # with its own power iteration
    lj, torch, ctx = env
    spec = [(24, 0.1), (37, 0.2), (48, 0.1), (31, 0.3)]
    probs = [adr_neumann(n, alpha=a, beta=-1.0, rate=100.0, seed=50 + i, amp=0.02) for i, (n, a) in enumerate(spec)]
    hs = [10.0 * p.h_cfl for p in probs]
    vs = [h * Operator(p).rhs(p.state) for p, h in zip(probs, hs)]
    b, ws, _ = make_batch(lj, torch, ctx, probs, hs, vs)
    b.run()
    rc, sts = b.stats()
    assert rc == 0
    for i, (p, h, v) in enumerate(zip(probs, hs, vs)):
        wo, so = phi_vertical(Operator(p), v, LS, AS, h, TOL)
        st = sts[i]
        say("batch adr vs oracle", i, p.nx, st["m_star"], so.m_star, "s", st["substeps"], so.substeps,
            "rej", st["rejections"], so.rejections, "iters", st["iters_total"], so.iters_total)
        assert abs(st["bound"] - so.bound) <= 1e-12 * so.bound
        assert st["m_star"] == so.m_star and st["substeps"] == so.substeps
        for k in range(3):
            assert rel(ws[i][k].cpu().numpy(), wo[k]) <= TOL
    b.close()


def test_batch_own_power_iteration(env):
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    b, ws, _ = make_batch(lj, torch, ctx, probs, hs, vs)
    b.run()
    rc, sts = b.stats()
    assert rc == 0
    for i, (p, h, v) in enumerate(zip(probs, hs, vs)):
        op = Operator(p)
        lam = power_iteration(op.jv, p.n)
        st = sts[i]
        assert st["power_iters"] == 20
        assert abs(st["bound"] - lam) <= 1e-12 * lam
        wo, so = phi_vertical(op, v, LS, AS, h, TOL)
        say("batch own bound", i, st["m_star"], so.m_star)
        assert st["m_star"] == so.m_star
        for k in range(3):
            assert rel(ws[i][k].cpu().numpy(), wo[k]) <= TOL
    b.close()


def test_batch_schedules_agree_and_tuner_reports(env):
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    bounds = [power_iteration(Operator(p).jv, p.n) for p in probs]
    ref = None
    try:
        for sched in range(8):
            os.environ["LJ_BATCH_SCHEDULE"] = str(sched)
            b, ws, _ = make_batch(lj, torch, ctx, probs, hs, vs, bounds=bounds)
            info = b.info()
            say("schedule", sched, info["block_size"], info["team"])
            assert info["schedule"] == sched and info["block_size"] in (256, 512, 1024)
            assert info["team"] in (1, 2, 4, 8, 16)
            b.run()
            rc, sts = b.stats()
            assert rc == 0
            out = [[w.cpu().numpy() for w in wi] for wi in ws]
            ms = [s["m_star"] for s in sts]
            if ref is None:
                ref = (out, ms)
            else:
                assert ms == ref[1]
                for i in range(len(probs)):
                    for k in range(3):
                        assert rel(out[i][k], ref[0][i][k]) <= 1e-13
            b.close()
    finally:
        os.environ.pop("LJ_BATCH_SCHEDULE", None)
    # the tuner times every schedule once per batch shape, then reuses its choice
    probs2 = [allen_cahn_noise(n, 0.05, seed=4100 + n) for n in (17, 29, 41)]
    hs2 = [10.0 * p.h_cfl for p in probs2]
    vs2 = [h * Operator(p).rhs(p.state) for p, h in zip(probs2, hs2)]
    b1, _, _ = make_batch(lj, torch, ctx, probs2, hs2, vs2)
    i1 = b1.info()
    assert len(i1["tune_ms"]) == i1["nschedules"] == 8 and all(t > 0 for t in i1["tune_ms"])
    assert i1["tune_ms"][i1["schedule"]] == min(i1["tune_ms"])
    b2, _, _ = make_batch(lj, torch, ctx, probs2, hs2, vs2)
    i2 = b2.info()
    assert i2["schedule"] == i1["schedule"] and all(t == 0 for t in i2["tune_ms"])
    b1.close()
    b2.close()


def test_batch_graph_replays_are_identical(env):
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    b, ws, (ops, vd) = make_batch(lj, torch, ctx, probs, hs, vs)
    first = None
    for rep in range(3):
        scratch = torch.randn(1 << 16, dtype=torch.float64, device="cuda:0")
        (scratch * 2.0).sum().item()  # eager work between replays
        for wi in ws:
            for w in wi:
                w.fill_(float("nan"))
        b.run()
        rc, sts = b.stats()
        assert rc == 0
        out = [w.cpu().numpy().copy() for wi in ws for w in wi]
        say("replay", rep)
        if first is None:
            first = out
        else:
            for a, c in zip(out, first):
                assert np.array_equal(a, c)
    b.close()


def test_batch_rejection_falls_back_to_substeps(env):
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    probs, hs, vs = probs[:3], hs[:3], vs[:3]
    bounds = [power_iteration(Operator(p).jv, p.n) for p in probs]
    opt = lj.lj_default_options(max_points=12)
    b, ws, _ = make_batch(lj, torch, ctx, probs, hs, vs, bounds=bounds, opt=opt)
    b.run()
    rc, sts = b.stats()
    assert rc == 0
    for i, (p, h, v) in enumerate(zip(probs, hs, vs)):
        wo, so = phi_vertical(Operator(p), v, LS, AS, h, TOL, Options(bound=bounds[i], max_points=12))
        st = sts[i]
        say("fallback", i, st["m_star"], st["substeps"], so.m_star, so.substeps)
        assert so.rejections >= 1 and st["rejections"] == so.rejections
        assert st["converged"] and st["m_star"] == so.m_star and st["substeps"] == so.substeps
        assert st["iters_total"] == so.iters_total
        for k in range(3):
            assert rel(ws[i][k].cpu().numpy(), wo[k]) <= TOL
    b.close()


def make_batch_ls(lj, torch, ctx, probs, hs, vs, ls, bounds, opt):
    ops = [lj.operator_from(p, "cuda:0") for p in probs]
    vd = [torch.as_tensor(v, dtype=torch.float64, device="cuda:0").contiguous() for v in vs]
    ws = [[torch.empty_like(v) for _ in ls] for v in vd]
    b = lj.Batch(ctx, ops, vd, hs, ls, [1.0] * len(ls), TOL, ws, bounds=bounds, opt=opt)
    return b, ws


@pytest.mark.parametrize("ls", [[0, 2], [3, 1, 0, 2]])
def test_batch_substeps_inside_the_launch(env, ls):
    """Accumulators the shared basis rejects are substepped inside the graph
    launch (Sec. 2.2, last paragraph; the substep identity of phi_l): the
    exponential's chain (l = 0) and phi_l with s - 1 exponentials and
    combinations; substep counts, rejections, every Newton step and the
    results against the oracle."""
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    hs = [8 * h for h in hs]
    vs = [8 * v for v in vs]
    bounds = [power_iteration(Operator(p).jv, p.n) for p in probs]
    opt = lj.lj_default_options(max_points=30)
    b, ws = make_batch_ls(lj, torch, ctx, probs, hs, vs, ls, bounds, opt)
    for rep in range(2):  # a replay redoes the substeps from the same inputs
        b.run()
        rc, sts = b.stats()
        assert rc == 0
        nsub = 0
        for i, (p, h, v) in enumerate(zip(probs, hs, vs)):
            wo, so = phi_vertical(Operator(p), v, ls, [1.0] * len(ls), h, TOL, Options(bound=bounds[i], max_points=30))
            st = sts[i]
            say("batch substeps", ls, i, p.nx, st["m_star"], st["substeps"], st["rejections"], so.m_star, so.substeps,
                so.rejections)
            assert st["converged"] and so.converged
            assert st["m_star"] == so.m_star and st["substeps"] == so.substeps
            assert st["rejections"] == so.rejections and st["iters_total"] == so.iters_total
            nsub += sum(x > 1 for x in so.substeps)
            for k in range(len(ls)):
                assert rel(ws[i][k].cpu().numpy(), wo[k]) <= TOL
        assert nsub >= 4
    b.close()


def test_batch_without_substeps_reports_the_rejection(env):
    """max_substeps = 1: a rejected accumulator stays rejected (m* -1, one
    substep) and the batch reports non-convergence, as the oracle does."""
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    probs, hs, vs = probs[:2], hs[:2], vs[:2]
    bounds = [power_iteration(Operator(p).jv, p.n) for p in probs]
    opt = lj.lj_default_options(max_points=6, max_substeps=1)
    b, ws = make_batch_ls(lj, torch, ctx, probs, hs, vs, [1, 3], bounds, opt)
    b.run()
    rc, sts = b.stats()
    assert rc == lj.LJ_ENOTCONV
    for i, (p, h, v) in enumerate(zip(probs, hs, vs)):
        wo, so = phi_vertical(Operator(p), v, [1, 3], [1.0, 1.0], h, TOL,
                              Options(bound=bounds[i], max_points=6, max_substeps=1))
        st = sts[i]
        assert not so.converged and not st["converged"]
        assert st["m_star"] == so.m_star and st["substeps"] == so.substeps and st["rejections"] == so.rejections
    b.close()


def test_batch_invalid_arguments(env):
    lj, torch, ctx = env
    probs, hs, vs = small_set()
    probs, hs, vs = probs[:2], hs[:2], vs[:2]
    ops = [lj.operator_from(p, "cuda:0") for p in probs]
    vd = [torch.as_tensor(v, device="cuda:0").contiguous() for v in vs]
    ws = [[torch.empty_like(v) for _ in range(3)] for v in vd]
    with pytest.raises(lj.LejaError, match="alias"):
        lj.Batch(ctx, ops, vd, hs, LS, AS, TOL, [[vd[0], ws[0][1], ws[0][2]], ws[1]])
    with pytest.raises(lj.LejaError, match="tol"):
        lj.Batch(ctx, ops, vd, hs, LS, AS, -1.0, ws)
    with pytest.raises(lj.LejaError, match="l must be"):
        lj.Batch(ctx, ops, vd, hs, [1, 2, 7], AS, TOL, ws)
    adv = lj.Operator("advdiff", probs[1].nx, probs[1].ny, 1, probs[1].dx, probs[1].dy, (1.0, 0.0, 0.0), None)
    with pytest.raises(lj.LejaError, match="one family"):
        lj.Batch(ctx, [ops[0], adv], vd, hs, LS, AS, TOL, ws)


def test_batch_full_ensemble_matches_plain_path(env):
    """The 256-instance ensemble (sizes 128..512, eps log-uniform): every
    instance converges in the batch; a sample of instances is re-run by the
    plain path on the batch's bound (same m*, 1e-10), and the smallest sampled
    instance is checked against the oracle with its own power iteration."""
    lj, torch, ctx = env
    probs = batch_instances()
    hs = [10.0 * p.h_cfl for p in probs]
    vs = [h * Operator(p).rhs(p.state) for p, h in zip(probs, hs)]
    say("full batch create", sum(p.n for p in probs))
    b, ws, (ops, vd) = make_batch(lj, torch, ctx, probs, hs, vs)
    info = b.info()
    say("schedule", info)
    b.run()
    rc, sts = b.stats()
    # h = 10x the diffusive CFL step of each instance: for the smallest eps the
    # step is long enough that the reaction eigenvalue +1 (outside the
    # interval) defeats the unsubstepped expansion, which the batch rejects and
    # substeps inside the launch
    assert rc == 0 and all(s["converged"] for s in sts)
    rejected = [i for i, s in enumerate(sts) if s["rejections"] > 0]
    say("rejected instances", len(rejected))
    assert len(rejected) >= 1
    # The rejected instances are those whose reaction eigenvalue +1 lies
    # outside the interval: an attempt at s substeps passes the hump test or
    # not by the rounding of its divided differences (pinned on the CPU:
    # test_batch_rejection_regime_is_rounding_decided), so the substep count
    # may differ between two correct FP64 runs.  Unique, and checked on the
    # smallest rejected instances: the plain GPU path on the batch's bound
    # takes exactly the batch's decisions; the oracle forced to the batch's
    # substep count reproduces its point counts and results to 1e-10; the
    # oracle's own choice of s is within a factor 2 and its result within
    # 10 (s + s') tol.
    for i in sorted(rejected, key=lambda j: probs[j].n)[:2]:
        st = sts[i]
        wp = [torch.empty_like(vd[i]) for _ in range(3)]
        rcp, sp = lj.lj_phi_vertical(ctx, ops[i], vd[i], LS, AS, hs[i], TOL, wp,
                                     lj.lj_default_options(bound=st["bound"]))
        assert rcp == 0
        for key in ("m_star", "substeps", "rejections", "iters_total"):
            assert sp[key] == st[key], key
        s_g = max(st["substeps"])
        wf, sf = phi_vertical(Operator(probs[i]), vs[i], LS, AS, hs[i], TOL,
                              Options(bound=st["bound"], substeps=s_g, max_substeps=s_g))
        wo, so = phi_vertical(Operator(probs[i]), vs[i], LS, AS, hs[i], TOL, Options(bound=st["bound"]))
        say("rejected vs oracle", i, probs[i].nx, st["m_star"], st["substeps"], "forced", sf.m_star,
            "own", so.m_star, so.substeps)
        assert sf.converged and sf.m_star == st["m_star"] and sf.substeps == st["substeps"]
        s_o = max(so.substeps)
        assert so.converged and s_o // 2 <= s_g <= 2 * s_o
        for k in range(3):
            w = ws[i][k].cpu().numpy()
            assert rel(w, wp[k].cpu().numpy()) <= TOL
            assert rel(w, wf[k]) <= TOL
            assert rel2(w, wo[k]) <= 10 * (s_g + s_o) * TOL
    sizes = np.array([p.nx for p in probs])
    sample = [int(np.flatnonzero(sizes == n)[j]) for n in (128, 192, 256, 384, 512) for j in (0, 1)]
    for i in sample:
        wp = [torch.empty_like(vd[i]) for _ in range(3)]
        rcp, sp = lj.lj_phi_vertical(ctx, ops[i], vd[i], LS, AS, hs[i], TOL, wp,
                                     lj.lj_default_options(bound=sts[i]["bound"]))
        say("plain vs batch", i, probs[i].nx, sp["m_star"], sts[i]["m_star"])
        assert rcp == 0 and sp["m_star"] == sts[i]["m_star"]
        for k in range(3):
            assert rel(ws[i][k].cpu().numpy(), wp[k].cpu().numpy()) <= TOL
    i = sample[0]
    op = Operator(probs[i])
    wo, so = phi_vertical(op, vs[i], LS, AS, hs[i], TOL)
    assert abs(sts[i]["bound"] - so.bound) <= 1e-12 * so.bound
    assert sts[i]["m_star"] == so.m_star
    for k in range(3):
        assert rel(ws[i][k].cpu().numpy(), wo[k]) <= TOL
    b.close()
