"""Brute-force twin of the oracle for tiny inputs, in arbitrary-precision Python.

TEST INFRASTRUCTURE ONLY.  Independent of ``oracle.c``: integers are Python ints reduced
with an explicit ``% 2**32`` and a two's-complement conversion; floating point is exact
rational arithmetic (``fractions.Fraction``) followed by an explicit round-to-nearest-even
to binary32, found by bracketing the candidate with its two binary32 neighbours.
"""
from fractions import Fraction
import math

import numpy as np

_TWO32 = 2 ** 32
# Smallest magnitude that rounds to infinity in binary32 (halfway between the largest
# finite value and 2^128).
_F32_MAX = Fraction(int(np.finfo(np.float32).max))
_F32_OVERFLOW = _F32_MAX + Fraction(2 ** 103, 2)


def to_i32(v):
    """Reduce an integer modulo 2^32 and read it as two's complement."""
    v %= _TWO32
    return v - _TWO32 if v >= 2 ** 31 else v


def affine_sum(x, a, b):
    y = [to_i32(a * xi + b) for xi in x]
    return y, sum(y)


def isum(x):
    return sum(int(v) for v in x)


def _bits(f):
    return int(np.float32(f).view(np.uint32))


def round_f32(q):
    """Round the exact rational q to binary32, round-to-nearest, ties to even."""
    if q == 0:
        return np.float32(0.0)
    if abs(q) >= _F32_OVERFLOW:
        return np.float32(math.copysign(math.inf, q))
    guess = np.float32(float(q)) if abs(q) <= _F32_MAX else np.float32(math.copysign(float(_F32_MAX), q))
    cands = {guess, np.nextafter(guess, np.float32(np.inf)), np.nextafter(guess, np.float32(-np.inf))}
    best = None
    for c in cands:
        if not np.isfinite(c):
            continue
        d = abs(Fraction(float(c)) - q)
        key = (d, _bits(c) & 1)   # nearer first, then the even significand
        if best is None or key < best[0]:
            best = (key, c)
    return np.float32(best[1])


def fma_f32(a, x, y):
    """One binary32 fused multiply-add a*x + y with a single rounding (finite inputs)."""
    a, x, y = np.float32(a), np.float32(x), np.float32(y)
    exact = Fraction(float(a)) * Fraction(float(x)) + Fraction(float(y))
    if exact == 0:
        # IEEE 754 sign of an exact zero sum under round-to-nearest: -0 only when both
        # the product and the addend are -0 (or negative zeros of equal sign).
        prod_neg = (math.copysign(1.0, float(a)) * math.copysign(1.0, float(x))) < 0
        y_neg = math.copysign(1.0, float(y)) < 0
        prod_zero = float(a) == 0.0 or float(x) == 0.0
        if prod_zero and float(y) == 0.0 and prod_neg and y_neg:
            return np.float32(-0.0)
        return np.float32(0.0)
    return round_f32(exact)


def saxpy(alpha, x, y):
    return [fma_f32(alpha, xi, yi) for xi, yi in zip(x, y)]


def slice_bounds(n, k, j):
    """Slice j of k: per-member length ceil(n/k) rounded up to a multiple of 256."""
    if k == 0 or j >= k:
        return n, n
    m = -(-n // k)
    m = -(-m // 256) * 256
    return min(n, j * m), min(n, (j + 1) * m)
