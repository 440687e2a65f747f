"""Pins of the variable-step oracle (Sec. 2.3): the cost controller's printed
constants, closed-form limits of both controllers, the invariants of an
integration (accepted estimates within tol, the end time hit exactly, the
retry size after a rejection), agreement with a fine classical RK4 solution,
and, for a linear problem (zero embedded estimate), the exact propagator."""
import math
import os

import numpy as np
import pytest

from oracle import adaptive as A
from oracle.exact import advdiff_symbol, fourier_closed_form
from oracle.integrators import rk_reference
from oracle.operators import Operator
from workloads import advdiff_bump, allen_cahn_noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cost_controller_constants.txt")


def test_constants_as_printed():
    vals = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    assert (A.ALPHA, A.BETA, A.LAMBDA, A.DELTA) == (vals["alpha"], vals["beta"], vals["lambda"], vals["delta"])


def test_cost_controller_limits():
    # equal sizes (D = 0): s = 1 lies in [1, lambda) -> grow by lambda
    assert A.cost_factor(0.1, 0.1, 5.0, 7.0) == A.LAMBDA
    # cost per unit time falling steeply as dt grows (D -> -inf): s -> e^alpha > lambda, taken as is
    g = A.cost_factor(2.0, 1.0, 1e-300, 1.0)
    assert g == pytest.approx(math.exp(A.ALPHA), rel=1e-12) and g > A.LAMBDA
    # rising steeply (D -> +inf): s -> e^-alpha < delta, taken as is
    g = A.cost_factor(2.0, 1.0, 1e300, 1.0)
    assert g == pytest.approx(math.exp(-A.ALPHA), rel=1e-12) and g < A.DELTA
    # slightly rising cost (0 < D small): s just below 1 -> shrink by delta
    assert A.cost_factor(2.0, 1.0, 1.01, 1.0) == A.DELTA
    # slightly falling: s just above 1 -> grow by lambda
    assert A.cost_factor(2.0, 1.0, 0.99, 1.0) == A.LAMBDA


def test_traditional_controller_closed_form():
    assert A.traditional_factor(1e-6, 1e-6, 3) == 1.0
    assert A.traditional_factor(16e-6, 1e-6, 3) == pytest.approx(0.5, rel=1e-15)
    assert A.traditional_factor(0.0, 1e-6, 3) == math.inf


@pytest.fixture(scope="module")
def ac_run():
    prob = allen_cahn_noise(32, eps=1e-2, seed=2, amp=0.5)
    T = 2.0 * prob.h_cfl
    run = A.integrate(prob, prob.state, T, prob.h_cfl, 1e-6, "EPIRK4S3", leja_tol=1e-12)
    return prob, T, run


def test_integration_invariants(ac_run):
    prob, T, run = ac_run
    assert run.t == T and run.accepted >= 3 and run.rejected >= 1
    acc = [a for a in run.attempts if a.accepted]
    assert all(a.err <= 1e-6 for a in acc)
    assert all(a.err > 1e-6 for a in run.attempts if not a.accepted)
    assert math.isclose(sum(a.dt for a in acc), T, rel_tol=1e-12)
    for a, b in zip(run.attempts, run.attempts[1:]):
        if not a.accepted:  # the retry uses the traditional size and starts at the same time
            assert b.t == a.t
            assert b.dt == pytest.approx(0.9 * a.dt * (1e-6 / a.err) ** 0.25, rel=1e-14)
    assert run.products == sum(a.cost for a in run.attempts)


def test_matches_fine_rk4(ac_run):
    prob, T, run = ac_run
    ref = rk_reference(lambda w: Operator(prob, state=w), prob.state, T, 2000)
    err = np.linalg.norm(run.u - ref) / np.linalg.norm(ref)
    assert err <= 10 * 1e-6 * run.accepted


def test_linear_problem_is_exact():
    """Advection-diffusion: f is linear, every remainder vanishes, so each step
    is the exact propagator and the embedded estimate is zero; only the cost
    controller sets the sizes."""
    prob, v = advdiff_bump()
    T = 6.0 * prob.h_cfl
    run = A.integrate(prob, v, T, prob.h_cfl, 1e-6, "EPIRK4S3", leja_tol=1e-13)
    acc = [a for a in run.attempts if a.accepted]
    assert run.rejected == 0 and all(a.err <= 1e-12 for a in acc)
    assert acc[1].dt == pytest.approx(A.LAMBDA * acc[0].dt, rel=1e-14)
    sig = advdiff_symbol(prob.nx, prob.ny, prob.dx, prob.dy, *prob.coef)
    exact = fourier_closed_form(sig, v, 0, T)
    assert np.linalg.norm(run.u - exact) / np.linalg.norm(exact) <= 1e-10 * len(acc) * 10
