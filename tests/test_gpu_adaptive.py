"""GPU parity of variable-step integration (lj_integrate, Sec. 2.3) with the
oracle's controller on the same seeded inputs: the same accepted and rejected
attempts, step sizes and Jacobian-product counts, and the same u(T); the
linear case against its exact propagator; argument errors."""
import numpy as np
import pytest

from gpu_util import GpuRunner, rel, rel2, say
from oracle import adaptive as A
from oracle.exact import advdiff_symbol, fourier_closed_form
from workloads import advdiff_bump, allen_cahn_noise, brusselator_perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    r = GpuRunner()
    yield r
    r.ctx.close()


def _gpu_integrate(gpu, prob, u0, T, dt0, tol, scheme, leja_tol, **kw):
    op = gpu.op(prob, state=u0)
    out = gpu.torch.empty_like(op.state)
    rc, st, recs = gpu.lj.lj_integrate(gpu.ctx, scheme, op, T, dt0, tol, leja_tol, out, **kw)
    gpu.torch.cuda.synchronize()
    return rc, st, recs, out.cpu().numpy()


def _compare(gpu, prob, u0, T, dt0, tol, scheme, leja_tol):
    orc = A.integrate(prob, u0, T, dt0, tol, scheme, leja_tol=leja_tol)
    rc, st, recs, u = _gpu_integrate(gpu, prob, u0, T, dt0, tol, scheme, leja_tol)
    say(prob.kind, scheme, "accepted/rejected", orc.accepted, orc.rejected, st["accepted"], st["rejected"],
        "products", orc.products, st["products"])
    assert rc == 0 and st["t"] == T
    assert (st["accepted"], st["rejected"]) == (orc.accepted, orc.rejected)
    assert st["products"] == orc.products
    assert len(recs) == len(orc.attempts)
    for r, a in zip(recs, orc.attempts):
        assert r["accepted"] == a.accepted and r["products"] == a.cost
        assert r["t"] == pytest.approx(a.t, rel=1e-9, abs=1e-300)
        assert r["dt"] == pytest.approx(a.dt, rel=1e-6)
        if a.accepted:
            assert r["err"] == pytest.approx(a.err, rel=1e-3)
    assert rel(u, orc.u) <= 1e-9
    return orc, st


def test_allen_cahn_epirk4s3_matches_oracle(gpu):
    prob = allen_cahn_noise(32, eps=1e-2, seed=2, amp=0.5)
    orc, _ = _compare(gpu, prob, prob.state, 2.0 * prob.h_cfl, prob.h_cfl, 1e-6, "EPIRK4S3", 1e-12)
    assert orc.rejected >= 1  # the first size is too large: a rejection and a retry


def test_allen_cahn_lekry_matches_oracle(gpu):
    # the LeKry form of EPIRK4s3: the third stage by Krylov, its products
    # counted in the cost controller's cost
    prob = allen_cahn_noise(32, eps=1e-2, seed=2, amp=0.5)
    _compare(gpu, prob, prob.state, 2.0 * prob.h_cfl, prob.h_cfl, 1e-6, "EPIRK4S3_LEKRY", 1e-12)
    _compare(gpu, prob, prob.state, 2.0 * prob.h_cfl, prob.h_cfl, 1e-6, "EPIRK4S3A", 1e-12)


def test_brusselator_exprb43_matches_oracle(gpu):
    prob = brusselator_perturbed(16, D=2e-2, seed=3, amp=0.3)
    _compare(gpu, prob, prob.state, 20.0 * prob.h_cfl, 2.0 * prob.h_cfl, 1e-5, "EXPRB43", 1e-12)


def test_linear_problem_exact_propagator(gpu):
    prob, v = advdiff_bump()
    T = 6.0 * prob.h_cfl
    rc, st, recs, u = _gpu_integrate(gpu, prob, v, T, prob.h_cfl, 1e-6, "EPIRK4S3", 1e-13)
    assert rc == 0 and st["rejected"] == 0 and st["t"] == T
    assert recs[1]["dt"] == pytest.approx(A.LAMBDA * recs[0]["dt"], rel=1e-14)
    sig = advdiff_symbol(prob.nx, prob.ny, prob.dx, prob.dy, *prob.coef)
    exact = fourier_closed_form(sig, v, 0, T)
    assert rel2(u, exact) <= 1e-9


def test_attempt_limit_and_arguments(gpu):
    prob = allen_cahn_noise(32, eps=1e-2, seed=2, amp=0.5)
    T = 2.0 * prob.h_cfl
    rc, st, recs, u = _gpu_integrate(gpu, prob, prob.state, T, prob.h_cfl, 1e-6, "EPIRK4S3", 1e-12, max_attempts=3)
    assert rc == gpu.lj.LJ_ENOTCONV and 0.0 < st["t"] < T and len(recs) == 3
    op = gpu.op(prob)
    out = gpu.torch.empty_like(op.state)
    lj = gpu.lj
    with pytest.raises(lj.LejaError, match="embedded scheme"):
        lj.lj_integrate(gpu.ctx, "EXPRB2", op, T, 0.1, 1e-6, 1e-10, out)
    with pytest.raises(lj.LejaError, match="dt0"):
        lj.lj_integrate(gpu.ctx, "EPIRK4S3", op, T, 0.0, 1e-6, 1e-10, out)
    with pytest.raises(lj.LejaError, match="alias"):
        lj.lj_integrate(gpu.ctx, "EPIRK4S3", op, T, 0.1, 1e-6, 1e-10, op.state)
    # T = 0: nothing to do, u_out = u(0)
    rc, st, recs = lj.lj_integrate(gpu.ctx, "EPIRK4S3", op, 0.0, 0.1, 1e-6, 1e-10, out)
    gpu.torch.cuda.synchronize()
    assert rc == 0 and st["accepted"] == 0 and np.array_equal(out.cpu().numpy(), prob.state)
