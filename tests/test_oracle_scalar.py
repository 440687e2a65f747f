"""Pins of the oracle's scalar parts: Leja points, phi_l, divided differences,
SplitMix64.  Each check compares against something other than the oracle's own
formula (exact values, brute force, an independent identity or library routine).
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg

from oracle.divdiff import divided_differences, newton_eval
from oracle.exact import phi_scalar_expm
from oracle.phi import phi, phi_mp
from oracle.points import leja_points
from oracle.splitmix import power_start_vector, splitmix64, uniform01

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- Leja points
def test_leja_first_points_exact(xi101):
    # xi_0 = 2 (start), xi_1 = -2, xi_2 = 0 are exact; xi_3 ties at +-2/sqrt(3),
    # the leftmost is taken.
    assert xi101[0] == 2.0 and xi101[1] == -2.0 and xi101[2] == 0.0
    assert abs(xi101[3] - (-2.0 / math.sqrt(3.0))) <= 4 * np.spacing(1.2)


def test_leja_points_are_brute_force_maximisers(xi101):
    # Every xi_m maximises prod_{j<m} |x - xi_j| on [-2, 2]: no point of a fine
    # uniform grid does better (brute force, independent of the gap search).
    grid = np.linspace(-2.0, 2.0, 200_001)
    acc = np.zeros_like(grid)
    for m in range(1, 101):
        with np.errstate(divide="ignore"):
            acc += np.log(np.abs(grid - xi101[m - 1]))
        best_grid = acc.max()
        at_xi = float(np.sum(np.log(np.abs(xi101[m] - xi101[:m]))))
        assert at_xi >= best_grid - 1e-9 * max(1.0, abs(best_grid)), m


def test_leja_points_distinct_in_interval(xi101):
    assert len(set(xi101.tolist())) == 101
    assert np.all(np.abs(xi101) <= 2.0)


def test_leja_points_golden(xi101):
    with open(os.path.join(GOLDEN, "leja_points_101.txt")) as fh:
        vals = [float.fromhex(s) for s in fh.read().split("\n") if s and not s.startswith("#")]
    assert np.array_equal(np.asarray(vals), xi101)


# ---------------------------------------------------------------------- phi_l
ZS = [-2000.0, -137.25, -37.5, -3.0, -1.0, -0.999, -0.5, -1e-3, -1e-9, 0.0, 1e-6, 0.3, 0.999, 1.0, 1.001, 2.0]


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_phi_integral_representation(l):
    # phi_l(z) = int_0^1 e^{(1-t) z} t^{l-1}/(l-1)! dt for l >= 1; phi_0 = exp.
    for z in ZS:
        got = phi(l, z)
        with mp.workdps(40):
            if l == 0:
                ref = mp.exp(z)
            else:
                ref = mp.quad(lambda t: mp.exp((1 - t) * z) * t ** (l - 1), [0, 0.5, 1]) / mp.factorial(l - 1)
        assert abs(got - float(ref)) <= 2e-16 * abs(float(ref)) + 1e-300, (l, z)


def test_phi_special_values():
    for l in range(6):
        assert phi(l, 0.0) == 1.0 / math.factorial(l)
    for z in [-50.0, -1.5, -1e-5, 0.7, 3.0]:
        assert abs(phi(0, z) - math.exp(z)) <= 1e-15 * math.exp(z)
        assert abs(phi(1, z) - math.expm1(z) / z) <= 4e-16 * abs(phi(1, z))


@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_phi_matches_augmented_expm(l):
    # Sec. 2.1 theorem on a 1x1 matrix, evaluated by scipy's Pade expm
    for z in [-300.0, -20.0, -2.0, -0.9, -0.01, 0.5, 1.5]:
        ref = phi_scalar_expm(l, z).real
        assert abs(phi(l, z) - ref) <= 1e-13 * abs(ref), (l, z)


def test_phi_complex_argument():
    for l in [0, 1, 3]:
        for z in [-3.0 + 4.0j, -0.2 + 0.5j, -100.0 - 60.0j]:
            ref = phi_scalar_expm(l, z)
            assert abs(phi(l, z) - ref) <= 1e-12 * abs(ref)


def test_phi_recurrence_across_branch():
    # series branch (|z| < 1) and recurrence branch (|z| >= 1) agree with
    # phi_l(z) = z phi_{l+1}(z) + 1/l!  on both sides of |z| = 1
    with mp.workdps(80):
        for z in [-1.0000001, -0.9999999, 0.9999999, 1.0000001]:
            for l in range(4):
                lhs = phi_mp(l, z)
                rhs = z * phi_mp(l + 1, z) + mp.mpf(1) / mp.factorial(l)
                assert abs(lhs - rhs) < mp.mpf(10) ** -60


# --------------------------------------------------------- divided differences
def test_divdiff_reproduces_polynomials(xi101):
    # DD of a degree-k polynomial: d_k = leading coefficient, d_m = 0 for m > k
    rng = np.random.default_rng(0)
    for k in [0, 1, 3, 6]:
        c = rng.uniform(-1, 1, size=k + 1)
        f = np.polyval(c, xi101[:20])
        d = divided_differences(f, xi101[:20])
        assert abs(d[k] - c[0]) <= 1e-12
        assert np.all(np.abs(d[k + 1:]) <= 1e-11)


def test_divdiff_newton_form_interpolates(xi101):
    f = [phi(1, -40.0 * (1.0 + 0.5 * x)) for x in xi101[:60]]
    d = divided_differences(f, xi101[:60])
    for j in range(60):
        assert abs(newton_eval(d, xi101, xi101[j]) - f[j]) <= 1e-13


@pytest.mark.parametrize("l", [0, 1, 3])
def test_divdiff_opitz(l, xi101):
    # Opitz: the divided differences of g at nodes xi are the first column of
    # g(Z), Z lower bidiagonal with the nodes on the diagonal and ones below it.
    # Here g(xi) = phi_l(s (c + gamma xi)); g(Z) e_0 via the augmented expm.
    M = 61
    s, c, gamma = 1.0, -30.0, 15.0
    Z = np.diag(xi101[:M]) + np.diag(np.ones(M - 1), -1)
    A = s * (c * np.eye(M) + gamma * Z)
    e0 = np.zeros(M)
    e0[0] = 1.0
    if l == 0:
        ref = scipy.linalg.expm(A)[:, 0]
    else:
        from oracle.exact import phi_dense
        ref = phi_dense(A, e0, l)
    f = [phi(l, s * (c + gamma * x)) for x in xi101[:M]]
    d = divided_differences(f, xi101[:M])
    scale = max(abs(x) for x in f)
    assert np.max(np.abs(d - ref)) <= 1e-12 * scale


def test_divdiff_fp64_vs_high_precision(xi101):
    # brute force: the same table in 100-digit arithmetic from 100-digit phi values;
    # FP64 error stays at round-off level relative to max|f| (Sec. 2.2 warns of it)
    M = 101
    for (l, s) in [(0, 50.0), (1, 100.0), (3, 100.0)]:
        c, gamma = -1.0, 0.5  # nodes s*(c + gamma*xi) span [-2s, 0]
        f64 = [phi(l, s * (c + gamma * x)) for x in xi101[:M]]
        d64 = divided_differences(f64, xi101[:M])
        with mp.workdps(100):
            xs = [mp.mpf(float(x)) for x in xi101[:M]]
            d = [phi_mp(l, s * (c + gamma * x), dps=100) for x in xs]
            for k in range(1, M):
                for j in range(M - 1, k - 1, -1):
                    d[j] = (d[j] - d[j - 1]) / (xs[j] - xs[j - k])
            err = max(abs(float(d[j]) - d64[j]) for j in range(M))
        assert err <= 1e-13 * max(abs(x) for x in f64), (l, s, err)


# ------------------------------------------------------------------ SplitMix64
def test_splitmix64_published_vectors():
    # reference outputs of the published generator
    assert splitmix64(0, 1)[0] == 0xE220A8397B1DCDAF
    assert splitmix64(1234567, 5) == [6457827717110365317, 3203168211198807973,
                                      9817491932198370423, 4593380528125082431,
                                      16408922859458223821]


def test_splitmix_uniform_vectorised_matches_stream():
    seed = 0x5EED
    ints = splitmix64(seed, 1000)
    u = uniform01(seed, 1000)
    assert np.array_equal(u, np.array([(z >> 11) * 2.0 ** -53 for z in ints]))
    x0 = power_start_vector(1000, seed)
    assert np.all((x0 >= 0.5) & (x0 < 1.5))
