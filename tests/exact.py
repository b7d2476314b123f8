"""Exact-arithmetic helpers for the oracle's pins (test-only)."""
from fractions import Fraction

import numpy as np


def round_to_f32(q: Fraction) -> float:
    """Round a rational to the nearest binary32 value (ties to even), exactly."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)                        # subnormal range keeps the -149 quantum
    quantum = Fraction(2) ** (e - 23)
    m = a / quantum
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * float(fl * quantum)


def f(x) -> Fraction:
    return Fraction(float(x))
