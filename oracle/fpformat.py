"""Exact round-to-nearest-even into small binary floating-point formats.

Oracle helper (test infrastructure only).  Rounding is done in exact rational
arithmetic straight from the FP64 value, so there is a single rounding and no
double rounding through an intermediate format.

A format is given by its number of stored mantissa bits and its minimum normal
exponent; values beyond the largest finite number overflow (reported as None).
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction

# (stored mantissa bits, minimum normal exponent, maximum exponent)
BINARY16 = (10, -14, 15)
BFLOAT16 = (7, -126, 127)


def max_finite(fmt) -> float:
    man, _emin, emax = fmt
    return float((2 - Fraction(1, 2 ** man)) * Fraction(2) ** emax)


def round_rne(x: float, fmt):
    """Nearest value of the format to x (ties to even); None on overflow."""
    if x == 0.0 or math.isnan(x):
        return x
    if math.isinf(x):
        return None
    man, emin, _emax = fmt
    m, e = math.frexp(x)          # x = m * 2**e, 0.5 <= |m| < 1
    exp = e - 1                   # x = 1.f * 2**exp
    q_exp = max(exp, emin) - man  # quantum of the binade (subnormals share emin's)
    q = Fraction(x) / (Fraction(2) ** q_exp)
    n = round(q)                  # Fraction.__round__ rounds half to even
    r = n * (Fraction(2) ** q_exp)
    if abs(r) > Fraction(max_finite(fmt)):
        return None
    v = float(r)
    if v == 0.0:
        return math.copysign(0.0, x)
    return v


def f16_bits(v: float) -> int:
    """binary16 bit pattern of a value that is exactly representable."""
    return struct.unpack("<H", struct.pack("<e", v))[0]


def bf16_bits(v: float) -> int:
    """bfloat16 bit pattern of a value that is exactly representable."""
    b = struct.unpack("<I", struct.pack("<f", v))[0]
    assert b & 0xFFFF == 0, "value not representable in bfloat16"
    return b >> 16


def bf16_value(bits: int) -> float:
    return struct.unpack("<f", struct.pack("<I", (bits & 0xFFFF) << 16))[0]


def f16_value(bits: int) -> float:
    return struct.unpack("<e", struct.pack("<H", bits & 0xFFFF))[0]
