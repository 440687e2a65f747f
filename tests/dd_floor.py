"""The rounding floor of the FP64 divided differences (Sec. 2.2, last
paragraph: with many Leja points the divided differences lose accuracy).

Near the stop index of a long expansion the FP64 table's high-order entries
can carry percent-level rounding error while their terms are still ~tol
||p||, so two correct FP64 implementations whose tables round differently
(another exp, another summation order) differ by about as much as either
differs from the same expansion with exact coefficients.  dd_floor() measures
that distance for the oracle: the oracle's action against the oracle's action
with every divided-difference table replaced by 60-digit values (mpmath,
phi_l from its definition), rounded to FP64.  A parity bar then reads
rel(gpu, oracle) <= tol + 2 dd_floor."""
import mpmath as mp
import numpy as np

import oracle.leja as leja


def _phi_mp(l, z):
    if z == 0:
        return 1 / mp.factorial(l)
    s = mp.e ** z
    for k in range(l):
        s -= z ** k / mp.factorial(k)
    return s / z ** l


def exact_coefficients(l, a, tau, c, gamma, npts):
    """coefficients() with 60-digit node values and table, rounded to FP64."""
    xi = leja.xi_table(max(npts, 101))[:npts]
    with mp.workdps(60):
        s = mp.mpf(a) * mp.mpf(tau)
        xs = [mp.mpf(float(x)) for x in xi]
        f = [_phi_mp(l, s * (mp.mpf(c) + mp.mpf(gamma) * x)) for x in xs]
        d = list(f)
        for k in range(1, npts):
            for j in range(npts - 1, k - 1, -1):
                d[j] = (d[j] - d[j - 1]) / (xs[j] - xs[j - k])
        return np.array([float(x) for x in d]), float(max(abs(x) for x in f))


def dd_floor(monkeypatch, run, metric):
    """metric(run() with FP64 tables, run() with exact tables); run() must
    call the oracle and return its result."""
    w64 = run()
    monkeypatch.setattr(leja, "coefficients", exact_coefficients)
    try:
        wex = run()
    finally:
        monkeypatch.undo()
    return metric(w64, wex)
