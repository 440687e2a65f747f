"""SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used as a counter-based generator for the
power-iteration start vector.

The i-th output (i = 0, 1, ...) of the stream seeded with `seed` is the mix
function applied to the state seed + (i+1) * 0x9E3779B97F4A7C15 (mod 2^64):

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

A uniform double in [0, 1) is (z >> 11) * 2^-53.  The HIP library implements
the same published generator on its own so that both sides draw the same start
vector without passing it in.
"""
from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def splitmix64(seed: int, count: int) -> list[int]:
    """First `count` outputs of SplitMix64 seeded with `seed` (Python ints)."""
    out = []
    state = seed & MASK
    for _ in range(count):
        state = (state + GOLDEN) & MASK
        z = state
        z = ((z ^ (z >> 30)) * M1) & MASK
        z = ((z ^ (z >> 27)) * M2) & MASK
        out.append(z ^ (z >> 31))
    return out


def uniform01(seed: int, n: int) -> np.ndarray:
    """U_i = (splitmix64 output i >> 11) * 2^-53 for i < n, vectorised in uint64."""
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK) + i * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def power_start_vector(n: int, seed: int) -> np.ndarray:
    """x_0[i] = 0.5 + U_i: the default power-iteration start vector."""
    return 0.5 + uniform01(seed, n)
