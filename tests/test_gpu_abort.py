"""Failure handling of the grid barrier, forced from the host: with the test
hook LJ_FORCE_SPIN_LIMIT the first (ordinary) launch of every action bounds
each barrier wait by a few polls, gives up, ends with its status marked
aborted, and the library repeats the action with a cooperative launch.  Every
kernel still exits normally; the results must equal those of a context
without the hook, bit for bit (the same deterministic arithmetic runs again)."""
import os

import numpy as np
import pytest

from gpu_util import say
from workloads import allen_cahn_noise, brusselator_perturbed

pytestmark = pytest.mark.gpu


def _run(lj, torch, ctx, prob, l, scheme=None):
    op = lj.operator_from(prob, "cuda:0")
    f = torch.empty_like(op.state)
    lj.lj_rhs(ctx, op, op.state, f)
    h = 10 * prob.h_cfl
    v = (h * f).contiguous()
    w = torch.empty_like(v)
    rc, st = lj.lj_phi_action(ctx, op, v, w, l, h, 1e-10)
    u_out = torch.empty_like(v)
    rcs, sts = lj.lj_step(ctx, scheme, op, h, 1e-10, u_out) if scheme else (0, None)
    torch.cuda.synchronize()
    return rc, st, w.cpu().numpy(), rcs, sts, u_out.cpu().numpy()


@pytest.mark.parametrize("name", ["tiled", "stream"])
def test_forced_barrier_abort_is_retried(name, monkeypatch):
    import torch

    import paper_2211_08948_amd as lj
    prob = allen_cahn_noise(256, eps=1e-3, seed=2) if name == "tiled" else brusselator_perturbed(256, D=2e-3, seed=3)
    ref_ctx = lj.Context(0)
    ref = _run(lj, torch, ref_ctx, prob, 1, "EPIRK4S3")
    ref_ctx.close()
    monkeypatch.setenv("LJ_FORCE_SPIN_LIMIT", "2")
    ctx = lj.Context(0)
    monkeypatch.delenv("LJ_FORCE_SPIN_LIMIT")
    lj.lj_timing_read(ctx, reset=True)
    got = _run(lj, torch, ctx, prob, 1, "EPIRK4S3")
    aborts = lj.lj_timing_read(ctx, reset=True)["aborts"]
    ctx.close()
    say("forced abort", name, "aborted launches", aborts, ref[1]["m_star"], got[1]["m_star"])
    assert aborts >= 2  # the action's and the step's first launches gave up
    assert got[0] == ref[0] == 0 and got[3] == ref[3] == 0
    assert got[1]["m_star"] == ref[1]["m_star"] and got[1]["bound"] == ref[1]["bound"]
    assert np.array_equal(got[2], ref[2])
    assert [s["m_star"] for s in got[4]] == [s["m_star"] for s in ref[4]]
    assert np.array_equal(got[5], ref[5])


def _krylov(lj, torch, ctx, prob):
    op = lj.operator_from(prob, "cuda:0")
    f = torch.empty_like(op.state)
    lj.lj_rhs(ctx, op, op.state, f)
    w = torch.empty_like(f)
    rc, st = lj.lj_phi_combination(ctx, op, [None, f, None, f], 10 * prob.h_cfl, 1e-10, w)
    torch.cuda.synchronize()
    return rc, st, w.cpu().numpy()


def test_forced_barrier_abort_krylov_basis(monkeypatch):
    """The persistent Krylov basis launch under the same hook: aborted, then
    repeated cooperatively, bit for bit the unhooked result."""
    import torch

    import paper_2211_08948_amd as lj
    prob = allen_cahn_noise(256, eps=1e-3, seed=2)
    ref_ctx = lj.Context(0)
    ref = _krylov(lj, torch, ref_ctx, prob)
    ref_ctx.close()
    monkeypatch.setenv("LJ_FORCE_SPIN_LIMIT", "2")
    ctx = lj.Context(0)
    monkeypatch.delenv("LJ_FORCE_SPIN_LIMIT")
    lj.lj_timing_read(ctx, reset=True)
    got = _krylov(lj, torch, ctx, prob)
    aborts = lj.lj_timing_read(ctx, reset=True)["aborts"]
    ctx.close()
    say("forced abort krylov", aborts, ref[1]["substeps"], got[1]["substeps"])
    assert aborts >= 1
    assert got[0] == ref[0] == 0 and got[1]["substeps"] == ref[1]["substeps"]
    assert got[1]["iters_total"] == ref[1]["iters_total"]
    assert np.array_equal(got[2], ref[2])
