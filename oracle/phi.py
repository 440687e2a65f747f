"""Scalar phi-functions (Sec. 1): phi_0(z) = e^z and
phi_{l+1}(z) = (phi_l(z) - 1/l!) / z, with phi_l(0) = 1/l!.

Reading: the paper prints the recurrence "for l >= 1"; it must hold from l = 0
on (phi_1(z) = (e^z - 1)/z is the function every integrator of Sec. 5 uses).

The oracle evaluates the definition in 80-digit arithmetic (mpmath) and rounds
once to FP64, so the FP64 value is correct to the last bit or so.  For |z| < 1
the equivalent Taylor series phi_l(z) = sum_k z^k / (k+l)! is summed instead of
the recurrence, only because the recurrence cancels there; at 80 digits either
form would do.
"""
from __future__ import annotations

import mpmath as mp

_DPS = 80


def phi_mp(l: int, z, dps: int = _DPS):
    """phi_l(z) as an mpmath number (real or complex z)."""
    if l < 0:
        raise ValueError("l must be >= 0")
    with mp.workdps(dps):
        zz = mp.mpmathify(z)
        if zz == 0:
            return mp.mpf(1) / mp.factorial(l)
        if abs(zz) < 1:
            # sum_k z^k/(k+l)!  until the terms fall below 10^-dps
            term = mp.mpf(1) / mp.factorial(l)
            total = term
            k = 0
            eps = mp.mpf(10) ** (-dps)
            while abs(term) > eps * abs(total):
                k += 1
                term = term * zz / (k + l)
                total += term
            return +total
        p = mp.exp(zz)
        for k in range(l):
            p = (p - mp.mpf(1) / mp.factorial(k)) / zz
        return +p


def phi(l: int, z) -> float | complex:
    """phi_l(z) rounded to FP64 (complex z gives a Python complex)."""
    v = phi_mp(l, z)
    if isinstance(v, mp.mpc):
        return complex(v)
    return float(v)


def phi_array(l: int, zs) -> "list[float]":
    """phi_l at every entry of zs (a sequence of real floats)."""
    return [phi(l, float(z)) for z in zs]
