"""Newton divided differences (Sec. 2.2: the interpolation coefficients d_m of
phi(Delta t (c + gamma xi)) at the Leja points are "determined using the divided
differences algorithm", Sec. 2.2, last paragraph).

Reading: the standard recursive table in FP64 on the normalised nodes xi_j of
[-2, 2] (never on the spectrum interval itself):

    d^(0)_j = f_j,
    d^(k)_j = (d^(k-1)_j - d^(k-1)_{j-1}) / (xi_j - xi_{j-k}),   j >= k,

and the coefficients are d_m = d^(m)_m.
"""
from __future__ import annotations

import numpy as np


def divided_differences(f, xi) -> np.ndarray:
    """Newton coefficients d_0..d_M of the data f_j at nodes xi_j (j = 0..M), FP64."""
    d = np.array(f, dtype=np.float64).copy()
    x = np.asarray(xi, dtype=np.float64)[: len(d)]
    M = len(d) - 1
    for k in range(1, M + 1):
        # right-hand side is evaluated from the previous column before assignment
        d[k:] = (d[k:] - d[k - 1:-1]) / (x[k:] - x[:-k])
    return d


def newton_eval(d, xi, x: float) -> float:
    """Value of the Newton-form polynomial sum_m d_m prod_{j<m} (x - xi_j) at x."""
    total = 0.0
    basis = 1.0
    for m in range(len(d)):
        total += d[m] * basis
        basis *= x - xi[m]
    return total
