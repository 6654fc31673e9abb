"""Exact-rational arithmetic and IEEE 754 rounding written from the standard's
definitions, used only to pin the oracle (it shares no code with `oracle/`).

round_fraction rounds an exact rational to binary32 / binary64 with
round-to-nearest, ties-to-even, gradual underflow and overflow to infinity.
"""
from __future__ import annotations

import math
from decimal import Decimal, localcontext
from fractions import Fraction

import numpy as np

FMT = {"f32": (24, -126, 127, np.float32), "f64": (53, -1022, 1023, np.float64)}


def floor_log2(a: Fraction) -> int:
    e = a.numerator.bit_length() - a.denominator.bit_length()
    two = Fraction(2)
    while two ** e > a:
        e -= 1
    while two ** (e + 1) <= a:
        e += 1
    return e


def round_fraction(q: Fraction, dtype: str, neg_zero: bool = False):
    """Nearest-even rounding of an exact rational to the format (returns a numpy scalar)."""
    p, emin, emax, t = FMT[dtype]
    if q == 0:
        return t(-0.0) if neg_zero else t(0.0)
    s = -1 if q < 0 else 1
    a = abs(q)
    e = max(floor_log2(a), emin)
    quantum = Fraction(2) ** (e - p + 1)
    n = a / quantum
    fl = n.numerator // n.denominator
    rem = n - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * quantum
    if r >= Fraction(2) ** (emax + 1):
        return t(s * math.inf)
    val = t(float(r))           # r is representable: exact conversion
    if val == 0:
        return t(-0.0) if s < 0 else t(0.0)
    return t(s * val)


def exact_sqrt_rounded(a: Fraction, dtype: str):
    """Correctly rounded square root of a non-negative rational."""
    p, emin, emax, t = FMT[dtype]
    if a == 0:
        return t(0.0)
    e = max(floor_log2(a) // 2, emin)
    quantum = Fraction(2) ** (e - p + 1)
    z = a / (quantum * quantum)
    n = math.isqrt(z.numerator // z.denominator)
    half = Fraction(2 * n + 1, 2)
    if z > half * half or (z == half * half and n % 2 == 1):
        n += 1
    return t(float(n * quantum))


def exp_rounded(x: float, dtype: str):
    """exp(x) from an 80-digit Decimal, rounded exactly."""
    if math.isnan(x):
        return FMT[dtype][3](math.nan)
    if x == -math.inf:
        return FMT[dtype][3](0.0)
    if x == math.inf:
        return FMT[dtype][3](math.inf)
    with localcontext() as ctx:
        ctx.prec = 80
        ctx.Emin = -10 ** 6
        ctx.Emax = 10 ** 6
        v = Decimal(x).exp()
    return round_fraction(Fraction(v), dtype)


def binop(op: str, a, b, dtype: str):
    """Correctly rounded a (op) b for finite binary values (IEEE semantics incl. signed zero)."""
    fa, fb = Fraction(float(a)), Fraction(float(b))
    if op == "add":
        q = fa + fb
        nz = (q == 0) and math.copysign(1, float(a)) < 0 and math.copysign(1, float(b)) < 0
    elif op == "sub":
        q = fa - fb
        nz = (q == 0) and math.copysign(1, float(a)) < 0 and math.copysign(1, float(b)) > 0 and fa == 0 and fb == 0
    elif op == "schur":
        q = fa * fb
        nz = (q == 0) and (math.copysign(1, float(a)) * math.copysign(1, float(b)) < 0)
    elif op == "div":
        if fb == 0:
            raise ZeroDivisionError
        q = fa / fb
        nz = (q == 0) and (math.copysign(1, float(a)) * math.copysign(1, float(b)) < 0)
    else:
        raise ValueError(op)
    return round_fraction(q, dtype, neg_zero=nz)


def ulp_distance(a, b) -> np.ndarray:
    """Distance in units in the last place between two float arrays of one dtype.

    Bit patterns are mapped to a monotone integer line (+0 and -0 both to 0);
    NaN vs NaN counts 0, NaN vs a number counts 2^62.
    """
    a = np.asarray(a)
    b = np.asarray(b)
    if a.dtype != b.dtype:
        raise TypeError("dtype mismatch")
    if a.dtype == np.float32:
        ia = a.view(np.int32).astype(np.int64)
        ib = b.view(np.int32).astype(np.int64)
        mask = np.int64(0x7FFFFFFF)
    else:
        ia = a.view(np.int64)
        ib = b.view(np.int64)
        mask = np.int64(0x7FFFFFFFFFFFFFFF)
    ma = np.where(ia < 0, -(ia & mask), ia).astype(np.longdouble)
    mb = np.where(ib < 0, -(ib & mask), ib).astype(np.longdouble)
    d = np.abs(ma - mb).astype(np.float64)
    nan_a, nan_b = np.isnan(a), np.isnan(b)
    d = np.where(nan_a & nan_b, 0.0, d)
    d = np.where(nan_a ^ nan_b, 2.0 ** 62, d)
    return d
