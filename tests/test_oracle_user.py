"""Pins of the oracle parts behind the user-operator path: the 1-D semilinear
problem of Sec. 3 (its exact solution, the discretisation, and the schemes'
convergence to the exact solution), and the finite-difference Jacobian
product (closed forms for linear and quadratic right-hand sides)."""
import math

import numpy as np
import pytest

from oracle.fdjac import SQRT_EPS, FDOperator, fd_step
from oracle.integrators import step
from oracle.leja import Options
from oracle.operators import Operator
from oracle.power import power_iteration
from oracle.semilinear import Semilinear, integrate_fixed
from workloads import advdiff_bump, burgers_sines


# ------------------------------------------------------------- semilinear (Sec. 3)
def test_simpson_weights_integrate_quadratics_exactly():
    # Simpson's rule is exact for cubics; both integrands vanish at x = 0 and 1
    p = Semilinear(31)
    assert abs(p.w @ (p.x * (1 - p.x)) - 1 / 6) <= 1e-16
    assert abs(p.w @ (p.x * p.x * (1 - p.x)) - 1 / 12) <= 1e-16


def test_exact_solution_solves_the_semi_discrete_system():
    # u = x(1-x)e^t sampled on the grid: f(u, t) = (x(1-x)e^t, 1) up to rounding
    p = Semilinear(31)
    for t in (0.0, 0.3, 1.0):
        U = p.exact(t)
        r = p.rhs(U)
        # the second difference of x(1-x) is -2 up to rounding of O(eps / dx^2)
        assert np.max(np.abs(r[:-1] - p.x * (1 - p.x) * math.exp(t))) <= 1e-11 * math.exp(t)
        assert r[-1] == 1.0


def test_jacobian_matches_dense_assembly():
    # J = [[D2 + 1 w^T, e^tau g], [0, 0]] assembled from its parts
    rng = np.random.default_rng(3)
    p = Semilinear(15)
    U = np.concatenate((rng.uniform(0, 1, 15), [0.4]))
    op = Semilinear(15, U)
    n = 16
    A = np.zeros((n, n))
    D2 = (np.diag(-2 * np.ones(15)) + np.diag(np.ones(14), 1) + np.diag(np.ones(14), -1)) / p.dx ** 2
    A[:15, :15] = D2 + np.outer(np.ones(15), p.w)
    A[:15, 15] = math.exp(0.4) * p.g
    J = np.column_stack([op.jv(e) for e in np.eye(n)])
    assert np.max(np.abs(J - A)) <= 1e-12 * np.max(np.abs(A))
    # and J is the derivative of f (f is linear in u and exponential in tau)
    v = rng.standard_normal(n)
    for eps in (1e-4,):
        fd = (op.rhs(U + eps * v) - op.rhs(U - eps * v)) / (2 * eps)
        assert np.linalg.norm(fd - op.jv(v)) <= 1e-6 * np.linalg.norm(op.jv(v))


def _oracle_step(op, scheme, h, tol, bound):
    return step(op, scheme, h, tol, Options(bound=bound))


@pytest.mark.parametrize("scheme", ["EXPRB43", "EPIRK4S3", "EPIRK4S3A"])
def test_schemes_converge_to_the_exact_solution(scheme):
    # end-to-end: the error at t = 1 is the integrator's alone and falls with
    # order ~4 (both schemes are fourth order) as the step is halved
    N = 31
    exact = Semilinear(N).exact(1.0)
    errs = []
    for nsteps in (4, 8):
        U, logs = integrate_fixed(N, scheme, 1.0, nsteps, 1e-11, _oracle_step,
                                  lambda op: power_iteration(op.jv, op.n, 20))
        assert all(b.converged for log in logs for b in log)
        errs.append(np.linalg.norm(U - exact) / np.linalg.norm(exact))
    order = math.log2(errs[0] / errs[1])
    assert errs[1] < 1e-5 and 3.5 <= order <= 5.0, (errs, order)


# --------------------------------------------------- finite-difference products
def test_fd_step_formula():
    u = np.array([3.0, 4.0])  # ||u|| = 5
    v = np.array([0.0, 2.0])
    assert fd_step(u, v) == SQRT_EPS * 6.0 / 2.0
    assert fd_step(u, np.zeros(2)) == 0.0
    assert np.all(FDOperator(Operator(advdiff_bump()[0], state=np.zeros(1024))).jv(np.zeros(1024)) == 0.0)


def test_fd_product_of_a_linear_rhs_is_exact_up_to_rounding():
    p, v = advdiff_bump()
    u = np.random.default_rng(1).uniform(-1, 1, p.n)
    fd = FDOperator(Operator(p, state=u))
    ref = Operator(p).jv(v)
    # rounding of f at u + eps v, divided by eps: ~ 2^-52 ||f(u)|| / (eps ||Jv||)
    assert np.linalg.norm(fd.jv(v) - ref) <= 1e-6 * np.linalg.norm(ref)


def test_fd_product_of_a_quadratic_rhs_has_the_closed_form_error():
    # Burgers at u = 0: f(e v) = e nu Lap v - (e^2 / 2)(d_x + d_y)(v^2), so the
    # forward difference is J v - (e/2)(d_x + d_y)(v^2), with f(0) = 0 exactly
    # (no cancellation: the rounding stays at 1e-16 of the terms)
    from oracle.operators import ddx, ddy
    p = burgers_sines(64, nu=1e-2, seed=5)
    p.state = np.zeros(p.n)
    op = Operator(p)
    v = np.random.default_rng(2).standard_normal(p.n)
    fd = FDOperator(op)
    e = fd_step(p.state, v)
    expect = op.jv(v) - 0.5 * e * (ddx(v * v, p.nx, p.ny, p.dx) + ddy(v * v, p.nx, p.ny, p.dy))
    # rounding of the e-scaled terms: ~1e-12 of J v, a few 1e-6 of the difference
    assert np.linalg.norm(fd.jv(v) - expect) <= 1e-4 * np.linalg.norm(fd.jv(v) - op.jv(v))
    assert np.linalg.norm(fd.jv(v) - op.jv(v)) > 1e-11 * np.linalg.norm(op.jv(v))  # far above rounding (1e-16)
