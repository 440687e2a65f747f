"""The allocation-free entry point lj_phi_action_noalloc against
lj_phi_action through the C ABI: the same kernels on the same inputs, so the
results and statistics must be identical -- on two calls in a row, the second
on a smaller grid (the scratch array keeps the first call's contents), with
substeps in the second.  Sizes beyond the scratch array and the learned
proposal are argument errors."""
import numpy as np
import pytest

from gpu_util import say
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


def _run(lj, torch, ctx, fn, prob, l, h, **opt):
    J = lj.operator_from(prob, "cuda:0")
    from oracle.operators import Operator
    v = torch.as_tensor(h * Operator(prob).rhs(prob.state), device="cuda:0").contiguous()
    w = torch.full_like(v, float("nan"))
    rc, st = fn(ctx, J, v, w, l, h, TOL, lj.lj_default_options(**opt))
    torch.cuda.synchronize()
    return rc, st, w.cpu().numpy()


def test_noalloc_matches_allocating_entry_point(env):
    lj, torch, ctx = env
    cases = [
        (allen_cahn_noise(512, eps=1e-3, seed=2), 1, 10.0, {}),              # 256 LDS tiles
        (allen_cahn_noise(96, eps=2e-2, seed=2), 3, 500.0, {}),              # smaller; s = 1 rejected, substeps
        (allen_cahn_noise(64, eps=5e-2, seed=2), 0, 10.0, {"substeps": 3}),  # forced substeps of exp
    ]
    for prob, l, mult, opt in cases:
        h = mult * prob.h_cfl
        say("noalloc", prob.kind, prob.nx, l, mult, opt)
        rc0, st0, w0 = _run(lj, torch, ctx, lj.lj_phi_action_noalloc, prob, l, h, **opt)
        rc1, st1, w1 = _run(lj, torch, ctx, lj.lj_phi_action, prob, l, h, **opt)
        assert rc0 == rc1 == 0
        for key in ("m_star", "substeps", "iters_total", "rejections", "power_iters", "bound"):
            assert st0[key] == st1[key], key
        assert np.array_equal(w0, w1)
        if mult > 100:
            assert st0["rejections"] >= 1


def test_noalloc_rejects_beyond_its_limit(env):
    lj, torch, ctx = env
    n = 2048
    prob = allen_cahn_noise(n, eps=1e-3, seed=2)
    J = lj.operator_from(prob, "cuda:0")
    v = torch.zeros(n * n, dtype=torch.float64, device="cuda:0")
    w = torch.empty_like(v)
    # 2 + 4 vectors of 32 MiB: far beyond the scratch array
    with pytest.raises(lj.LejaError) as e:
        lj.lj_phi_action_noalloc(ctx, J, v, w, 1, prob.h_cfl, TOL, lj.lj_default_options())
    assert e.value.code == lj.LJ_EINVAL and "scratch" in str(e.value)
    small = allen_cahn_noise(32, eps=1e-2, seed=2)
    Js = lj.operator_from(small, "cuda:0")
    vs = torch.ones(32 * 32, dtype=torch.float64, device="cuda:0")
    ws = torch.empty_like(vs)
    with pytest.raises(lj.LejaError) as e:
        lj.lj_phi_action_noalloc(ctx, Js, vs, ws, 1, small.h_cfl, TOL, lj.lj_default_options(use_proposal=1))
    assert e.value.code == lj.LJ_EINVAL
    assert lj.LJ_NOALLOC_SCRATCH_BYTES == 32 << 20
