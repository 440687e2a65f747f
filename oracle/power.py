"""Power-iteration estimate of the largest eigenvalue magnitude of J
(Sec. 2.2: "a rough estimate of the spectrum ... can be obtained using power
iterations"; Sec. 5.1: its cost has to be counted).

Readings (the paper fixes none of these):
  * start vector x_0[i] = 0.5 + U_i, U_i the i-th SplitMix64 uniform of a seed
    (a constant start vector is an eigenvector of the periodic Laplacian and
    would stall);
  * a fixed number K of Jacobian products, no convergence-based stop;
  * the estimate is lambda = ||J x_{K-1}|| / ||x_{K-1}|| with x_k = J^k x_0
    (normalised after every product to stay in range; normalisation does not
    change the ratio).
"""
from __future__ import annotations

import numpy as np

from .splitmix import power_start_vector


def power_iteration(jv, n: int, iters: int = 20, seed: int = 0x5EED, x0=None) -> float:
    """lambda_hat = ||J x_{K-1}|| / ||x_{K-1}|| after K = iters products."""
    if iters < 1:
        raise ValueError("iters must be >= 1")
    x = power_start_vector(n, seed) if x0 is None else np.array(x0, dtype=np.float64)
    lam = 0.0
    for _ in range(iters):
        y = jv(x)
        nx = np.linalg.norm(x)
        ny = np.linalg.norm(y)
        lam = ny / nx
        if ny == 0.0:
            return 0.0
        x = y / ny
    return float(lam)
