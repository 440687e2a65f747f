"""The register-tiled kernel with several 32 x 32 tiles per block (grids of
more tiles than CUs): actions, the vertical form with accumulators that stop
inside a super-step (the commit from a snapshot or a rerun of the
super-step), power iteration, rejections with substeps and a scheme step,
against the oracle on the same seeded inputs; and against the streaming
kernel on the same inputs.  Sizes: 576^2 (324 tiles, one or two per block),
1024^2 (four per block) and a non-square 1024 x 320 advection-diffusion
grid; ragged grids (600^2, 1000 x 300: the last column and row of tiles
narrower) on the same kernel."""
import os

import numpy as np
import pytest

from gpu_util import GpuRunner, rel, say
from oracle.integrators import step as oracle_step
from oracle.leja import Options, phi_action, phi_vertical
from oracle.operators import Operator
from oracle.power import power_iteration
from workloads import allen_cahn_noise
from workloads.problems import Problem

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def gpu():
    r = GpuRunner()
    yield r
    r.ctx.close()


@pytest.fixture(scope="module")
def ac576():
    prob = allen_cahn_noise(576, eps=1e-3, seed=2)
    op = Operator(prob)
    return prob, op, power_iteration(op.jv, prob.n, 20)


@pytest.fixture(scope="module")
def ac1024():
    prob = allen_cahn_noise(1024, eps=1e-3, seed=2)
    op = Operator(prob)
    return prob, op, power_iteration(op.jv, prob.n, 20)


@pytest.mark.parametrize("l", [1, 3])
@pytest.mark.parametrize("mult", [1, 10])
def test_action_576(gpu, ac576, l, mult):
    prob, op, lam = ac576
    h = mult * prob.h_cfl
    v = h * op.rhs(prob.state)
    w_orc, st_orc = phi_action(op, v, l, h, TOL, Options(bound=lam))
    say("multi-tile 576", l, mult, st_orc.m_star)
    rc, st, w = gpu.action(prob, v, l, h, TOL, bound=lam)
    assert rc == 0 and st["m_star"] == st_orc.m_star
    assert rel(w, w_orc) <= TOL


def test_bound_and_vertical_1024(gpu, ac1024):
    prob, op, lam = ac1024
    say("multi-tile 1024 bound")
    lam_gpu = gpu.bound(prob, 20)
    assert abs(lam_gpu - lam) <= 1e-12 * lam
    h = 10 * prob.h_cfl
    v = h * op.rhs(prob.state)
    ls, As = [1, 1, 1], [1 / 8, 1 / 9, 1.0]
    ws_orc, st_orc = phi_vertical(op, v, ls, As, h, TOL, Options(bound=lam))
    say("multi-tile 1024 vertical", st_orc.m_star)
    assert min(st_orc.m_star) < 16 < max(st_orc.m_star)  # a stop inside the first super-step
    rc, st, ws = gpu.vertical(prob, v, ls, As, h, TOL, bound=lam)
    assert rc == 0 and st["m_star"] == st_orc.m_star
    for a, b in zip(ws, ws_orc):
        assert rel(a, b) <= TOL


def test_own_power_iteration_action_1024(gpu, ac1024):
    prob, op, lam = ac1024
    h = 10 * prob.h_cfl
    v = h * op.rhs(prob.state)
    w_orc, st_orc = phi_action(op, v, 2, h, TOL)
    rc, st, w = gpu.action(prob, v, 2, h, TOL)
    say("multi-tile 1024 own bound", st["bound"], st_orc.bound, st_orc.m_star)
    assert rc == 0 and st["power_iters"] == 20
    assert abs(st["bound"] - st_orc.bound) <= 1e-12 * st_orc.bound
    assert st["m_star"] == st_orc.m_star and rel(w, w_orc) <= TOL


def test_advdiff_nonsquare(gpu):
    nx, ny = 1024, 320
    dx = 1.0 / nx
    a = 1.0 / dx
    prob = Problem("advdiff", nx, ny, 1, dx, dx, (1.0, a, a), None, dx * dx / 4.0)
    op = Operator(prob)
    rng = np.random.default_rng(12)
    v = rng.standard_normal(prob.n)
    h = 10 * prob.h_cfl
    lam = power_iteration(op.jv, prob.n, 20)
    w_orc, st_orc = phi_action(op, v, 1, h, TOL, Options(bound=lam))
    say("multi-tile advdiff 1024x320", st_orc.m_star)
    rc, st, w = gpu.action(prob, v, 1, h, TOL, bound=lam)
    assert rc == 0 and st["m_star"] == st_orc.m_star
    assert rel(w, w_orc) <= TOL


def test_rejection_substeps_576(gpu, ac576):
    prob, op, lam = ac576
    h = 10 * prob.h_cfl
    v = h * op.rhs(prob.state)
    w_orc, st_orc = phi_action(op, v, 1, h, TOL, Options(bound=lam, max_points=14))
    say("multi-tile substeps", st_orc.substeps, st_orc.rejections, st_orc.iters_total)
    assert st_orc.rejections >= 1
    rc, st, w = gpu.action(prob, v, 1, h, TOL, bound=lam, max_points=14)
    assert rc == 0
    assert (st["substeps"], st["rejections"], st["iters_total"]) == \
        (st_orc.substeps, st_orc.rejections, st_orc.iters_total)
    assert rel(w, w_orc) <= TOL


def test_epirk4s3_step_576(gpu, ac576):
    prob, op, lam = ac576
    h = 10 * prob.h_cfl
    u_orc, e_orc, log = oracle_step(op, "EPIRK4S3", h, TOL)
    rc, sts, u_gpu, e_gpu = gpu.step(prob, "EPIRK4S3", h, TOL)
    say("multi-tile EPIRK4s3", [b.m_star for b in log])
    assert rc == 0
    for a, b in zip(sts, log):
        assert a["m_star"][:len(b.m_star)] == b.m_star
    assert rel(u_gpu - prob.state, u_orc - prob.state) <= TOL
    assert rel(e_gpu, e_orc) <= 1e-8


def test_multitile_matches_streaming_kernel(gpu, ac1024):
    """The same action through the streaming kernel (LJ_NO_REG=1 at context
    creation): identical point counts, results within 1e-12."""
    import paper_2211_08948_amd as lj
    prob, op, lam = ac1024
    h = 30 * prob.h_cfl
    v = h * op.rhs(prob.state)
    rc, st, w = gpu.action(prob, v, 1, h, TOL, bound=lam)
    os.environ["LJ_NO_REG"] = "1"
    try:
        ctx2 = lj.Context(0)
    finally:
        del os.environ["LJ_NO_REG"]
    try:
        J = gpu.op(prob)
        vd = gpu.dev(v)
        w2 = gpu.torch.empty_like(vd)
        rc2, st2 = lj.lj_phi_action(ctx2, J, vd, w2, 1, h, TOL, lj.lj_default_options(bound=lam))
        gpu.torch.cuda.synchronize()
        say("multi-tile vs streaming", st["m_star"], st2["m_star"])
        assert rc == rc2 == 0 and st["m_star"] == st2["m_star"]
        assert rel(w, w2.cpu().numpy()) <= 1e-12
    finally:
        ctx2.close()


@pytest.fixture(scope="module")
def ac600():
    # 600 = 18 * 32 + 24: 19 x 19 = 361 tiles (more than CUs), those of the
    # last column and row 24 points wide
    prob = allen_cahn_noise(600, eps=1e-3, seed=4)
    op = Operator(prob)
    return prob, op, power_iteration(op.jv, prob.n, 20)


def _tiled(gpu, fn):
    lj = gpu.lj
    lj.lj_timing_read(gpu.ctx, reset=True)
    lj.lj_timing_enable(gpu.ctx, True)
    try:
        out = fn()
    finally:
        lj.lj_timing_enable(gpu.ctx, False)
    tm = lj.lj_timing_read(gpu.ctx, reset=True)
    return out, tm


@pytest.mark.parametrize("l", [1, 2])
def test_ragged_600_action(gpu, ac600, l):
    prob, op, lam = ac600
    h = 10 * prob.h_cfl
    v = h * op.rhs(prob.state)
    w_orc, st_orc = phi_action(op, v, l, h, TOL, Options(bound=lam))
    say("ragged 600^2", l, st_orc.m_star)
    (rc, st, w), tm = _tiled(gpu, lambda: gpu.action(prob, v, l, h, TOL, bound=lam))
    assert tm["tiled_launches"] == tm["launches"] >= 1  # the register-tiled kernel ran
    assert rc == 0 and st["m_star"] == st_orc.m_star
    assert rel(w, w_orc) <= TOL


def test_ragged_600_vertical_own_bound(gpu, ac600):
    # the power iteration, a stop inside the first super-step (the commit from
    # a snapshot or a rerun) and four accumulators' instance on ragged tiles
    prob, op, lam = ac600
    h = 10 * prob.h_cfl
    v = h * op.rhs(prob.state)
    ls, As = [1, 1, 1], [1 / 8, 1 / 9, 1.0]
    ws_orc, st_orc = phi_vertical(op, v, ls, As, h, TOL)
    say("ragged 600^2 vertical", st_orc.m_star)
    assert min(st_orc.m_star) < 16 < max(st_orc.m_star)
    (rc, st, ws), tm = _tiled(gpu, lambda: gpu.vertical(prob, v, ls, As, h, TOL))
    assert tm["tiled_launches"] == tm["launches"] >= 1
    assert rc == 0 and st["m_star"] == st_orc.m_star
    assert abs(st["bound"] - st_orc.bound) <= 1e-12 * st_orc.bound
    for a, b in zip(ws, ws_orc):
        assert rel(a, b) <= TOL


def test_ragged_advdiff_nonsquare(gpu):
    # 1000 x 300: 32 x 10 = 320 tiles, the last column 8 wide, the last row 12 high
    nx, ny = 1000, 300
    dx = 1.0 / nx
    a = 1.0 / dx
    prob = Problem("advdiff", nx, ny, 1, dx, dx, (1.0, a, 0.5 * a), None, dx * dx / 4.0)
    op = Operator(prob)
    rng = np.random.default_rng(13)
    v = rng.standard_normal(prob.n)
    h = 10 * prob.h_cfl
    lam = power_iteration(op.jv, prob.n, 20)
    w_orc, st_orc = phi_action(op, v, 1, h, TOL, Options(bound=lam))
    say("ragged advdiff 1000x300", st_orc.m_star)
    (rc, st, w), tm = _tiled(gpu, lambda: gpu.action(prob, v, 1, h, TOL, bound=lam))
    assert tm["tiled_launches"] == tm["launches"] >= 1
    assert rc == 0 and st["m_star"] == st_orc.m_star
    assert rel(w, w_orc) <= TOL


def test_ragged_advdiff_vertical(gpu):
    # the four-accumulator instance on ragged tiles (1000 x 300, as above):
    # phi_1..phi_3 at a_k = 1/3, 1/2, 1 sharing one basis, with stops inside
    # a super-step, against the oracle
    nx, ny = 1000, 300
    dx = 1.0 / nx
    a = 1.0 / dx
    prob = Problem("advdiff", nx, ny, 1, dx, dx, (1.0, a, 0.5 * a), None, dx * dx / 4.0)
    op = Operator(prob)
    v = np.random.default_rng(14).standard_normal(prob.n)
    h = 10 * prob.h_cfl
    lam = power_iteration(op.jv, prob.n, 20)
    ls, As = [1, 2, 3], [1 / 3, 1 / 2, 1.0]
    ws_orc, st_orc = phi_vertical(op, v, ls, As, h, TOL, Options(bound=lam))
    say("ragged advdiff vertical", st_orc.m_star)
    (rc, st, ws), tm = _tiled(gpu, lambda: gpu.vertical(prob, v, ls, As, h, TOL, bound=lam))
    assert tm["tiled_launches"] == tm["launches"] >= 1
    assert rc == 0 and st["m_star"] == st_orc.m_star
    for x, y in zip(ws, ws_orc):
        assert rel(x, y) <= TOL


def test_ragged_matches_streaming_kernel(gpu, ac600):
    """The ragged grid through the streaming kernel (LJ_NO_REG=1 at context
    creation): identical point counts, results within 1e-12."""
    import paper_2211_08948_amd as lj
    prob, op, lam = ac600
    h = 30 * prob.h_cfl
    v = h * op.rhs(prob.state)
    rc, st, w = gpu.action(prob, v, 1, h, TOL, bound=lam)
    os.environ["LJ_NO_REG"] = "1"
    try:
        ctx2 = lj.Context(0)
    finally:
        del os.environ["LJ_NO_REG"]
    try:
        J = gpu.op(prob)
        vd = gpu.dev(v)
        w2 = gpu.torch.empty_like(vd)
        rc2, st2 = lj.lj_phi_action(ctx2, J, vd, w2, 1, h, TOL, lj.lj_default_options(bound=lam))
        gpu.torch.cuda.synchronize()
        say("ragged vs streaming", st["m_star"], st2["m_star"])
        assert rc == rc2 == 0 and st["m_star"] == st2["m_star"]
        assert rel(w, w2.cpu().numpy()) <= 1e-12
    finally:
        ctx2.close()
