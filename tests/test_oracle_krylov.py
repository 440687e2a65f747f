"""Pins of the Krylov evaluation of phi-function combinations (the horizontal
stage of LeKry) against dense Pade expm of the augmented matrix (Sec. 2.1
theorem), the Leja action, the Lanczos property of a symmetric J, and of the
LeKry step against EPIRK4s3 (the same scheme, stages evaluated differently)."""
import numpy as np
import pytest

from oracle.exact import phi_dense
from oracle.integrators import step
from oracle.krylov import KrylovOptions, arnoldi, phi_combination
from oracle.leja import Options, phi_action
from oracle.operators import Operator
from oracle.power import power_iteration
from workloads import advdiff_bump, allen_cahn_noise, brusselator_perturbed


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


def _dense_combination(J, bs, h):
    out = np.zeros(J.shape[0])
    for j, b in enumerate(bs):
        if b is not None:
            out += phi_dense(h * J, b, j) * h ** j
    return out


def _problems():
    ac = allen_cahn_noise(16, eps=1e-2, seed=8)
    ac.state = ac.state * 8
    return {"allencahn": ac, "advdiff": advdiff_bump(16)[0],
            "brusselator": brusselator_perturbed(12, D=0.1, seed=8, amp=0.3)}


@pytest.mark.parametrize("name", ["allencahn", "advdiff", "brusselator"])
@pytest.mark.parametrize("window", [2, 0])
def test_combination_matches_dense_pade(name, window):
    p = _problems()[name]
    op = Operator(p)
    J = op.dense()
    rng = np.random.default_rng(1)
    h = 10 * p.h_cfl
    bs = [rng.uniform(-1, 1, p.n), rng.uniform(-1, 1, p.n), None, rng.uniform(-1, 1, p.n), rng.uniform(-1, 1, p.n)]
    ref = _dense_combination(J, bs, h)
    for tol in (1e-10, 1e-13):
        w, st = phi_combination(op.jv, bs, h, tol, KrylovOptions(window=window))
        assert st.converged and rel(w, ref) <= 10 * tol + 1e-14, (tol, st)


def test_exponential_matches_leja_and_more_substeps_with_small_spaces():
    p = _problems()["allencahn"]
    op = Operator(p)
    h = 10 * p.h_cfl
    v = np.random.default_rng(2).uniform(-1, 1, p.n)
    ref = phi_dense(h * op.dense(), v, 0)
    w30, s30 = phi_combination(op.jv, [v], h, 1e-12)
    w8, s8 = phi_combination(op.jv, [v], h, 1e-12, KrylovOptions(m=8))
    wl, _ = phi_action(op, v, 0, h, 1e-12)
    # Krylov within its tolerance; Leja within the 10 tol its single-term estimate leaves (C.8)
    assert rel(w30, ref) <= 1e-11 and rel(w8, ref) <= 1e-11 and rel(wl, ref) <= 1e-10
    assert s8.substeps > s30.substeps


def test_symmetric_jacobian_window_two_is_lanczos():
    # J symmetric (Allen-Cahn): orthogonalising against the last two vectors
    # gives the same tridiagonal H as full orthogonalisation
    p = _problems()["allencahn"]
    op = Operator(p)
    v = np.random.default_rng(3).uniform(-1, 1, p.n)
    _, H2, m2, _, _ = arnoldi(op.jv, v, 12, 2)
    _, H0, m0, _, _ = arnoldi(op.jv, v, 12, 0)
    assert m2 == m0 == 12
    assert np.max(np.abs(H2 - np.triu(np.tril(H0, 1), -1))) <= 1e-8 * np.max(np.abs(H0))
    assert np.max(np.abs(np.triu(H0, 2))) <= 1e-8 * np.max(np.abs(H0))


def test_breakdown_gives_the_exact_result():
    # v an eigenvector of a diagonal J: the Krylov space is one-dimensional
    from workloads.problems import Problem
    lam = -np.linspace(1.0, 50.0, 40)
    p = Problem("diag", 40, 1, 1, 1.0, 1.0, (), lam, 1.0)
    op = Operator(p)
    v = np.zeros(40)
    v[7] = 2.0
    w, st = phi_combination(op.jv, [v], 0.3, 1e-12)
    assert st.products == 1 and abs(w[7] - 2.0 * np.exp(0.3 * lam[7])) <= 1e-13 * abs(w[7])
    assert np.count_nonzero(w) == 1


@pytest.mark.parametrize("base", ["EPIRK4S3", "EPIRK4S3A"])
def test_lekry_step_equals_epirk4s3(base):
    # the same scheme: u_4 and the embedded error agree within the tolerances
    p = allen_cahn_noise(48, eps=2e-2, seed=2)
    op = Operator(p)
    h = 10 * p.h_cfl
    lam = power_iteration(op.jv, p.n, 20)
    u_e, e_e, _ = step(op, base, h, 1e-12, Options(bound=lam))
    u_k, e_k, log = step(op, base + "_LEKRY", h, 1e-12, Options(bound=lam))
    assert len(log) == 3 and all(b.converged for b in log)
    assert rel(u_k, u_e) <= 1e-10 and rel(e_k, e_e) <= 1e-6
