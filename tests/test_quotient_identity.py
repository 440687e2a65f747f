"""The device kernels form t / den as q = t r, q + (t - q den) r with
r = 1/den and both corrections fused multiply-adds (Markstein's correction).
They rely on this being the correctly rounded quotient, i.e. the value of an
IEEE division; here the same arithmetic is carried out exactly on the host
(each FMA rounded once, through rational arithmetic) and compared with
Python's division on random and near-boundary operands."""
import random
from fractions import Fraction


def _fma(a: float, b: float, c: float) -> float:
    # one rounding of the exact a*b + c (int/int true division is correctly rounded)
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _div_rn(t: float, den: float) -> float:
    r = 1.0 / den
    q = t * r
    return _fma(_fma(-q, den, t), r, q)


def _mant(rng, lo=-20, hi=20):
    return rng.uniform(1.0, 2.0) * 2.0 ** rng.randint(lo, hi) * rng.choice((-1.0, 1.0))


def test_random_operands():
    rng = random.Random(1)
    for _ in range(150000):
        t, den = _mant(rng), _mant(rng)
        assert _div_rn(t, den) == t / den, (t.hex(), den.hex())


def test_quotients_near_binade_edges():
    """t chosen so that t / den sits just below or above a power of two times
    (1 - k 2^-52), where the product t r is furthest from the quotient in ulps."""
    import math
    rng = random.Random(2)
    for _ in range(150000):
        den = _mant(rng)
        target = 2.0 ** rng.randint(0, 9) * (1.0 - rng.randint(0, 999) * 2.0 ** -52)
        t = math.nextafter(den * target, rng.choice((math.inf, -math.inf)))
        assert _div_rn(t, den) == t / den, (t.hex(), den.hex())


def test_leja_step_like_operands():
    """Operands of the Newton step's quotient: gamma = 1.25 lam / 4 for spectral
    bounds over many decades, numerators over the range the basis takes."""
    rng = random.Random(3)
    for _ in range(20000):
        gamma = 1.25 * rng.uniform(1.0, 10.0) * 10.0 ** rng.randint(-2, 9) / 4.0
        t = rng.uniform(-1.0, 1.0) * gamma * 10.0 ** rng.randint(-3, 3)
        assert _div_rn(t, gamma) == t / gamma, (t.hex(), gamma.hex())
