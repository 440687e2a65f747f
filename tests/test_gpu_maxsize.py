"""Parity at the largest sizes, where the oracle cannot run the whole action:
outputs are checked at sampled points against closed forms that hold at any
size, computed by the oracle's pinned routines one point at a time.

* advection-diffusion on an 8192 x 8192 periodic grid (67M points, the
  largest grid of the measured sweep) from a sum of three Fourier modes: J
  acts by the stencil's symbol, so phi_1(hJ)v is the same sum with each
  amplitude times phi_1(h sigma_k); through the register-tiled kernel with
  several tiles per block (the default at this size) and through the
  streaming kernel (LJ_NO_TILE=1 at context creation);
* a diagonal operator of 2^28 entries (2 GiB per vector): w_i = phi_1(h
  lambda_i) v_i.

The Leja stop test bounds the 2-norm error relative to the result (~tol); the
sampled relative RMS error estimates it, and the largest sampled error is
bounded loosely as a guard against localised indexing mistakes."""
import os

import numpy as np
import pytest

from gpu_util import say
from oracle.exact import advdiff_symbol_at, phi_scalar_expm
from oracle.phi import phi
from workloads import diag_problem, fourier_modes, uniform_vector
from workloads.problems import Problem

pytestmark = pytest.mark.gpu
TOL = 1e-10
NSAMPLE = 200_000


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2211_08948_amd as lj
    ctx = lj.Context(0)
    yield lj, torch, ctx
    ctx.close()
    torch.cuda.empty_cache()


def _check(w_s, ref_s, what):
    err = w_s - ref_s
    rms = np.sqrt(np.mean(err ** 2)) / np.sqrt(np.mean(ref_s ** 2))
    mx = np.max(np.abs(err)) / np.max(np.abs(ref_s))
    say(what, "sampled relative rms error", rms, "max", mx)
    assert rms <= 10 * TOL
    assert mx <= 1e-7


@pytest.mark.parametrize("kernel", ["register", "stream"])
def test_advdiff_8192_fourier_modes(env, kernel):
    lj, torch, ctx = env
    if kernel == "stream":
        os.environ["LJ_NO_TILE"] = "1"
        try:
            ctx = lj.Context(0)
        finally:
            del os.environ["LJ_NO_TILE"]
    n, nu = 8192, 1.0
    dx = 1.0 / n
    a = nu / dx  # grid Peclet number 1
    prob = Problem("advdiff", n, n, 1, dx, dx, (nu, a, a), None, dx * dx / (4 * nu))
    v, modes = fourier_modes(n, 3, seed=11, kmax=40)
    h = 10 * prob.h_cfl
    say("advdiff 8192^2", kernel, modes)
    J = lj.operator_from(prob, "cuda:0")
    vd = torch.as_tensor(v, device="cuda:0")
    del v
    w = torch.empty_like(vd)
    lj.lj_timing_read(ctx, reset=True)
    lj.lj_timing_enable(ctx, True)
    rc, st = lj.lj_phi_action(ctx, J, vd, w, 1, h, TOL)
    torch.cuda.synchronize()
    lj.lj_timing_enable(ctx, False)
    tm = lj.lj_timing_read(ctx, reset=True)
    assert rc == 0 and st["converged"]
    assert tm["tiled_launches"] == (1 if kernel == "register" else 0)
    rng = np.random.default_rng(12)
    idx = rng.integers(0, n * n, size=NSAMPLE)
    jj, ii = np.divmod(idx, n)
    ref = np.zeros(NSAMPLE)
    for kx, ky, A, th in modes:
        sig = advdiff_symbol_at(2 * np.pi * kx / n, 2 * np.pi * ky / n, dx, dx, nu, a, a)
        ph = 2 * np.pi * (kx * ii + ky * jj) / n + th
        ref += (A * phi_scalar_expm(1, h * sig) * np.exp(1j * ph)).real
    w_s = w[torch.as_tensor(idx, device="cuda:0")].cpu().numpy()
    del vd, w
    if kernel == "stream":
        ctx.close()
    _check(w_s, ref, f"advdiff 8192^2 {kernel} m*={st['m_star']}")


def test_diag_2p28(env):
    lj, torch, ctx = env
    n = 1 << 28
    prob = diag_problem(n, -300.0, seed=13)
    v = uniform_vector(n, -1.0, 1.0, seed=14)
    h = 0.2
    J = lj.operator_from(prob, "cuda:0")
    vd = torch.as_tensor(v, device="cuda:0")
    w = torch.empty_like(vd)
    rc, st = lj.lj_phi_action(ctx, J, vd, w, 1, h, TOL)
    torch.cuda.synchronize()
    assert rc == 0 and st["converged"]
    rng = np.random.default_rng(15)
    idx = rng.integers(0, n, size=NSAMPLE // 4)
    ref = np.array([phi(1, h * prob.state[i]) * v[i] for i in idx])
    w_s = w[torch.as_tensor(idx, device="cuda:0")].cpu().numpy()
    del vd, w, J
    _check(w_s, ref, f"diag 2^28 m*={st['m_star']} bound={st['bound']:.2f}")
