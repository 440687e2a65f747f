"""The benchmarked workload at full size, run the way the benchmark runs it.

512^2 Allen-Cahn (eps = 1e-3, u0 ~ U[-0.1, 0.1] seed 2), tol 1e-10: EXPRB2 and
EPIRK4s3 steps (Sec. 5.1 equation) with default options -- the GPU's own
power iteration over the 256 tiles of the LDS-tiled kernel, the bound kept on
the device between the actions of a step, every launch of the step enqueued
back to back -- against the oracle's step with its own power iteration, at
1x, 10x and 100x the explicit diffusive step; the stand-alone phi_2 action
of the benchmark; and the power iteration started from a given vector
(lj_options.pi_start, lj_spectral_bound's start) against the oracle's."""
import numpy as np
import pytest

from gpu_util import GpuRunner, rel, say
from oracle.integrators import step as oracle_step
from oracle.leja import Options, phi_action
from oracle.operators import Operator
from oracle.power import power_iteration
from workloads import allen_cahn_noise, burgers_sines

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def gpu():
    r = GpuRunner()
    yield r
    r.ctx.close()


@pytest.fixture(scope="module")
def metric():
    prob = allen_cahn_noise(512, eps=1e-3, seed=2)
    op = Operator(prob)
    lam = power_iteration(op.jv, prob.n, 20)
    return prob, op, lam


def test_own_bound_512(gpu, metric):
    prob, op, lam = metric
    say("bound 512^2")
    lam_gpu = gpu.bound(prob, 20)
    assert abs(lam_gpu - lam) <= 1e-12 * lam


@pytest.mark.parametrize("mult", [1, 10, 100])
@pytest.mark.parametrize("scheme", ["EXPRB2", "EPIRK4S3"])
def test_step_parity_metric_config(gpu, metric, scheme, mult):
    prob, op, lam = metric
    h = mult * prob.h_cfl
    u = prob.state
    u_orc, e_orc, log = oracle_step(op, scheme, h, TOL)
    say("metric step", scheme, mult, [b.m_star for b in log])
    rc, sts, u_gpu, e_gpu = gpu.step(prob, scheme, h, TOL)
    assert rc == 0 and len(sts) == len(log)
    assert abs(sts[0]["bound"] - log[0].bound) <= 1e-12 * log[0].bound
    assert sts[0]["power_iters"] == log[0].power_iters == 20
    for a, b in zip(sts, log):
        K = len(b.m_star)
        assert a["m_star"][:K] == b.m_star and a["substeps"][:K] == b.substeps
        assert a["iters_total"] == b.iters_total and a["rejections"] == b.rejections
    # the step's increment carries the method's arithmetic; u itself is
    # dominated by the state
    assert rel(u_gpu - u, u_orc - u) <= TOL
    if e_orc is not None:
        # err = u_4 - u_3 is formed from two rounded vectors of the size of u
        assert np.max(np.abs(e_gpu - e_orc)) <= 1e-8 * np.max(np.abs(e_orc)) + 1e-13 * np.max(np.abs(u_orc))


@pytest.mark.parametrize("mult", [1, 10, 100])
def test_phi2_action_metric_config(gpu, metric, mult):
    # the benchmark's stand-alone phi_2(hJ) h f(u) on the step's bound
    prob, op, lam = metric
    h = mult * prob.h_cfl
    v = h * op.rhs(prob.state)
    w_orc, st_orc = phi_action(op, v, 2, h, TOL, Options(bound=lam))
    say("metric phi_2", mult, st_orc.m_star)
    rc, st, w = gpu.action(prob, v, 2, h, TOL, bound=lam)
    assert rc == 0 and st["m_star"] == st_orc.m_star and st["substeps"] == st_orc.substeps
    assert rel(w, w_orc) <= TOL


@pytest.mark.parametrize("n", [512, 96, 37])
def test_power_iteration_from_given_start(gpu, n):
    # lj_spectral_bound with a start vector, on the tiled (512^2, 96^2) and
    # the ragged grid, and on Burgers (streaming kernel), against the oracle
    # started from the same vector
    probs = [allen_cahn_noise(n, eps=1e-3 if n == 512 else 2e-2, seed=2)]
    if n == 96:
        probs.append(burgers_sines(96, nu=3e-2, seed=5))
    for prob in probs:
        op = Operator(prob)
        x0 = np.random.default_rng(31 + n).uniform(-1.0, 1.0, prob.n)
        for iters in (1, 7, 20):
            lam_orc = power_iteration(op.jv, prob.n, iters, x0=x0)
            say("pi_start", prob.kind, n, iters)
            lam_gpu = gpu.lj.lj_spectral_bound(gpu.ctx, gpu.op(prob), iters, start=gpu.dev(x0))
            assert abs(lam_gpu - lam_orc) <= 1e-12 * lam_orc


def test_action_with_pi_start_option(gpu):
    # lj_options.pi_start: the action's own power iteration starts from it
    prob = allen_cahn_noise(96, eps=2e-2, seed=2)
    op = Operator(prob)
    h = 10 * prob.h_cfl
    v = h * op.rhs(prob.state)
    x0 = np.random.default_rng(77).uniform(0.0, 1.0, prob.n)
    lam = power_iteration(op.jv, prob.n, 20, x0=x0)
    w_orc, st_orc = phi_action(op, v, 1, h, TOL, Options(bound=lam))
    say("pi_start option", lam)
    start = gpu.dev(x0)
    rc, st, w = gpu.action(prob, v, 1, h, TOL, pi_start=start)
    assert rc == 0 and st["power_iters"] == 20
    assert abs(st["bound"] - lam) <= 1e-12 * lam
    assert st["m_star"] == st_orc.m_star and rel(w, w_orc) <= TOL
    # a different start vector gives a (slightly) different bound: the option is used
    rc, st2, _ = gpu.action(prob, v, 1, h, TOL)
    assert st2["bound"] != st["bound"]
