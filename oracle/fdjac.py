"""Finite-difference Jacobian products -- TEST INFRASTRUCTURE (plain NumPy).

Sec. 4 computes the Jacobian-vector products numerically.  The reading here
(the paper gives no formula): a forward difference of the right-hand side,

    J(u) v ~ (f(u + eps v) - f(u)) / eps,  eps = sqrt(2^-52) (1 + ||u||_2) / ||v||_2,

the step length commonly used by Jacobian-free Newton-Krylov methods (Knoll
and Keyes 2004), f(u) evaluated once; J(u) 0 = 0.  Its error is
O(eps ||f''||) + O(2^-52 ||f|| / eps), about 1e-8 relative.
"""
from __future__ import annotations

import math

import numpy as np

SQRT_EPS = math.sqrt(2.0 ** -52)


def fd_step(u, v) -> float:
    nv = float(np.linalg.norm(v))
    if nv == 0.0:
        return 0.0
    return SQRT_EPS * (1.0 + float(np.linalg.norm(u))) / nv


class FDOperator:
    """An operator (rhs, state, n) whose jv is the forward difference of rhs."""

    def __init__(self, op):
        self.op = op
        self.state = np.asarray(op.state, dtype=np.float64)
        self.n = op.n
        self.fu = op.rhs(self.state)

    def rhs(self, x) -> np.ndarray:
        return self.op.rhs(x)

    def jv(self, v) -> np.ndarray:
        v = np.asarray(v, dtype=np.float64)
        eps = fd_step(self.state, v)
        if eps == 0.0:
            return np.zeros_like(v)
        return (self.op.rhs(self.state + eps * v) - self.fu) / eps

    def remainder(self, x, fu=None) -> np.ndarray:
        if fu is None:
            fu = self.fu
        return self.rhs(x) - fu - self.jv(np.asarray(x) - self.state)
