"""Exact reductions that close an expression (test infrastructure only).

accu (sum of all elements, Fig. 1 and Section 5 task 1), sum along a dimension,
dot and norm, defined as the exact sum of the real values that enter them; and
the further closing reductions min, max, mean, 1-norm and infinity norm (Armadillo
functions of the same names), from the same exact sums or the element values; and
the statistics mean and variance along a dimension and variance of all elements
(listed among the library's functions, Section 2), from exact sums as well.

* Floating types: each binary32 / binary64 value is an integer mantissa times a
  power of two.  Mantissas are summed per exponent in integer-exact arithmetic
  and the per-exponent totals are combined as Python integers, giving the exact
  rational sum (a Fraction).  `to_float` rounds it once for reporting.
* dot(x, y) sums the exact products x_i * y_i (a binary32 product is exact in
  binary64; binary64 products are formed from integer mantissas).
* norm(x) = sqrt(exact sum of x_i^2).
* Integer types: the sum reduced mod 2^32 (order-independent, so bit-exact).

Readings: accu(x % y) is dot(x, y) — the whole-expression
pattern matching of Section 3 applied to a reduction; sum(X, 0) is per column
(1 x n_cols), sum(X, 1) per row (n_rows x 1); the reduction of an empty operand is 0.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .elementwise import FLOATS, round_to


CHUNK = 1 << 25          # elements per exact-summation pass; keeps every bucket below 2^26


def _split_f64(x: np.ndarray):
    """x (float64 array, finite) -> (int64 mantissa m, int64 exponent e) with x = m * 2^e, |m| < 2^53.

    Read straight from the binary64 fields: biased exponent b and fraction f give
    m = 2^52 + f, e = b - 1075 for normal numbers and m = f, e = -1074 for subnormals.
    """
    bits = np.ascontiguousarray(x, dtype=np.float64).view(np.int64)
    b = (bits >> 52) & 0x7FF
    f = bits & ((1 << 52) - 1)
    normal = b > 0
    m = np.where(normal, f | (1 << 52), f)
    e = np.where(normal, b - 1075, -1074)
    m = np.where(bits < 0, -m, m)
    return m, e


def _bucket_sum(mant: np.ndarray, expo: np.ndarray, group: np.ndarray | None, n_groups: int):
    """Exact sum of mant * 2^expo per group, as a list of Fractions.

    Mantissas are split into a high and a low part of at most 27 bits each; per
    (group, exponent) the parts are summed in binary64, which is exact as long as
    the count per bucket stays below 2^26 (checked).
    """
    if group is None:
        group = np.zeros(mant.shape, dtype=np.int64)
    mant = mant.ravel()
    expo = expo.ravel()
    group = group.ravel()
    if mant.size and np.bincount(group).max() >= (1 << 26):
        raise ValueError("bucket too large for exact float64 accumulation")
    sign = np.where(mant < 0, -1, 1)
    am = np.abs(mant)
    hi = (am >> 27) * sign
    lo = (am & ((1 << 27) - 1)) * sign
    emin = int(expo.min()) if expo.size else 0
    eidx = expo - emin
    ne = int(eidx.max()) + 1 if expo.size else 1
    key = group * ne + eidx
    s_hi = np.bincount(key, weights=hi.astype(np.float64), minlength=n_groups * ne)
    s_lo = np.bincount(key, weights=lo.astype(np.float64), minlength=n_groups * ne)
    s_hi = s_hi.reshape(n_groups, ne)
    s_lo = s_lo.reshape(n_groups, ne)
    out = []
    for g in range(n_groups):
        nz = np.flatnonzero((s_hi[g] != 0) | (s_lo[g] != 0))
        tot = 0
        base = emin
        for j in nz:
            v = (int(s_hi[g, j]) << 27) + int(s_lo[g, j])
            tot += Fraction(v) * Fraction(2) ** (int(j) + base)
        out.append(Fraction(tot))
    return out


def _finite_or_raise(x):
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite value in an exact reduction")


def exact_sum(x: np.ndarray) -> Fraction:
    """Exact sum of a float32/float64 array (parity pinned: Fraction brute force, closed forms)."""
    x = np.asarray(x)
    if x.size == 0:
        return Fraction(0)
    flat = x.ravel()
    tot = Fraction(0)
    step = CHUNK
    for s in range(0, flat.size, step):
        x64 = flat[s:s + step].astype(np.float64)
        _finite_or_raise(x64)
        m, e = _split_f64(x64)
        tot += _bucket_sum(m, e, None, 1)[0]
    return tot


def exact_dot(x: np.ndarray, y: np.ndarray) -> Fraction:
    """Exact sum of x_i * y_i."""
    x = np.asarray(x).ravel()
    y = np.asarray(y).ravel()
    if x.shape != y.shape:
        raise ValueError("dot: length mismatch")
    if x.size == 0:
        return Fraction(0)
    if x.dtype in (np.float32, np.float16) and y.dtype in (np.float32, np.float16):
        p = x.astype(np.float64) * y.astype(np.float64)     # exact: at most 24 + 24 bits
        _finite_or_raise(p)
        return exact_sum(p)
    # binary64 operands: products from integer mantissas (4 partial products of <= 27 bits)
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    _finite_or_raise(x)
    _finite_or_raise(y)
    mx, ex = _split_f64(x)
    my, ey = _split_f64(y)
    sgn = np.sign(mx) * np.sign(my)
    ax, ay = np.abs(mx), np.abs(my)
    xh, xl = ax >> 26, ax & ((1 << 26) - 1)
    yh, yl = ay >> 26, ay & ((1 << 26) - 1)
    e = ex + ey
    tot = Fraction(0)
    step = CHUNK
    for a, b, sh in ((xh, yh, 52), (xh, yl, 26), (xl, yh, 26), (xl, yl, 0)):
        prod = (a * b) * sgn              # < 2^54: split again by _bucket_sum
        for s in range(0, prod.size, step):
            tot += _bucket_sum(prod[s:s + step].astype(np.int64), (e + sh)[s:s + step], None, 1)[0]
    return tot


def exact_sum_dim(X: np.ndarray, dim: int) -> list:
    """Exact per-column (dim 0 -> 1 x n_cols) or per-row (dim 1 -> n_rows x 1) sums, as Fractions."""
    X = np.asarray(X)
    r, c = X.shape
    if dim not in (0, 1):
        raise ValueError("dim must be 0 or 1")
    n_groups = c if dim == 0 else r
    if X.size == 0:
        return [Fraction(0)] * n_groups
    x64 = X.astype(np.float64)
    _finite_or_raise(x64)
    m, e = _split_f64(x64)
    if dim == 0:
        group = np.broadcast_to(np.arange(c, dtype=np.int64)[None, :], (r, c))
    else:
        group = np.broadcast_to(np.arange(r, dtype=np.int64)[:, None], (r, c))
    return _bucket_sum(m, e, np.ascontiguousarray(group), n_groups)


def to_float(q: Fraction) -> float:
    """Round an exact value once to binary64 (nearest-even; Fraction -> float is correctly rounded)."""
    return float(q)


def round_exact(q: Fraction, dtype: str) -> float:
    """An exact value rounded once to the element type (nearest-even), as a Python float.

    float() of a Fraction is correctly rounded to binary64; a second rounding to
    binary32 or a 16-bit type is innocuous (53 >= 2p + 2), so the result is the
    correctly rounded value of q in that type.
    """
    return float(round_to(np.float64(float(q)), dtype))


def sum_abs(x: np.ndarray) -> float:
    """sum |x_i| rounded to binary64 (the scale used when the exact sum is 0)."""
    return to_float(exact_sum(np.abs(np.asarray(x))))


# ---------------------------------------------------------------------------
# Closing reductions on the element type
# ---------------------------------------------------------------------------

def accu(x: np.ndarray, dtype: str):
    """Sum of all elements: exact Fraction for floats, int mod 2^32 (as the dtype's value) for integers."""
    x = np.asarray(x)
    if dtype in FLOATS:
        return exact_sum(x)
    u = x.astype(np.int64).astype(np.uint64) if dtype == "s32" else x.astype(np.uint64)
    tot = int(np.sum(u, dtype=np.uint64)) & 0xFFFFFFFF      # uint64 wraps mod 2^64 -> exact mod 2^32
    if dtype == "s32" and tot >= 1 << 31:
        tot -= 1 << 32
    return tot


def sum_dim(X: np.ndarray, dim: int, dtype: str):
    """Per-column / per-row sums; Fractions for floats, ints mod 2^32 for integers."""
    X = np.asarray(X)
    if dtype in FLOATS:
        return exact_sum_dim(X, dim)
    u = X.astype(np.int64).astype(np.uint64) if dtype == "s32" else X.astype(np.uint64)
    s = np.sum(u, axis=0 if dim == 0 else 1, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    out = [int(v) for v in s]
    if dtype == "s32":
        out = [v - (1 << 32) if v >= 1 << 31 else v for v in out]
    return out


def dot(x, y, dtype: str):
    if dtype not in FLOATS:
        raise ValueError("dot is defined here for floating types only")
    return exact_dot(x, y)


def norm(x, dtype: str) -> float:
    """Vector 2-norm (Frobenius for a matrix): sqrt of the exact sum of squares, in binary64.

    The exact sum is scaled by an even power of two before the square root so that
    neither the sum nor its root leaves the binary64 range.
    """
    if dtype not in FLOATS:
        raise ValueError("norm is defined here for floating types only")
    s = exact_dot(x, x)
    if s == 0:
        return 0.0
    k = (s.numerator.bit_length() - s.denominator.bit_length()) // 2
    scaled = s / Fraction(2) ** (2 * k)
    return math.ldexp(math.sqrt(float(scaled)), k)


# ---------------------------------------------------------------------------
# Further closing reductions (min, max, mean, 1-norm, infinity norm)
# ---------------------------------------------------------------------------

def _values(x, dtype):
    x = np.asarray(x).ravel()
    if x.size == 0:
        raise ValueError("min / max of an empty operand")
    return x


def vmax(x, dtype):
    """Largest element (an element value of the type).  NaN as soon as one element is
    NaN (the NaN-propagating maximum of IEEE 754-2019)."""
    x = _values(x, dtype)
    if dtype in FLOATS:
        x64 = x.astype(np.float64)
        if np.isnan(x64).any():
            return math.nan
        return float(x64.max())
    return int(x.astype(np.int64).max())


def vmin(x, dtype):
    """Smallest element, NaN-propagating like vmax."""
    x = _values(x, dtype)
    if dtype in FLOATS:
        x64 = x.astype(np.float64)
        if np.isnan(x64).any():
            return math.nan
        return float(x64.min())
    return int(x.astype(np.int64).min())


def mean(x, dtype) -> Fraction:
    """Exact mean: the exact sum divided by the element count (floating types)."""
    if dtype not in FLOATS:
        raise ValueError("mean is defined here for floating types only")
    x = np.asarray(x)
    if x.size == 0:
        raise ValueError("mean of an empty operand")
    return exact_sum(x) / x.size


def norm1(x, dtype) -> Fraction:
    """1-norm of the elements taken as a vector: the exact sum of |x_i|."""
    if dtype not in FLOATS:
        raise ValueError("norm1 is defined here for floating types only")
    return exact_sum(np.abs(np.asarray(x)))


def norm_inf(x, dtype) -> float:
    """Infinity norm of the elements taken as a vector: the largest |x_i| (0 for an empty
    operand), NaN as soon as one element is NaN."""
    if dtype not in FLOATS:
        raise ValueError("norm_inf is defined here for floating types only")
    x64 = np.abs(np.asarray(x).astype(np.float64)).ravel()
    if x64.size == 0:
        return 0.0
    if np.isnan(x64).any():
        return math.nan
    return float(x64.max())


# ---------------------------------------------------------------------------
# Statistics: mean along a dimension, variance (Section 2 lists mean and variance
# among the library's functions; the semantics are Armadillo's mean(X, dim) and
# var(X, norm_type, dim))
# ---------------------------------------------------------------------------

def mean_dim(X, dim: int, dtype: str) -> list:
    """Exact per-column (dim 0) or per-row (dim 1) means as Fractions; None where the
    count is 0 (the mean of no elements, 0 / 0, is NaN)."""
    if dtype not in FLOATS:
        raise ValueError("mean is defined here for floating types only")
    X = np.asarray(X)
    cnt = X.shape[0] if dim == 0 else X.shape[1]
    sums = exact_sum_dim(X, dim)
    return [None if cnt == 0 else q / cnt for q in sums]


def _sum_sq_dev(x: np.ndarray) -> Fraction:
    """Exact sum over the elements of (x_i - mu)^2, mu the exact mean.

    Expanding the square, sum (x_i - mu)^2 = sum x_i^2 - 2 mu sum x_i + n mu^2
    = sum x_i^2 - (sum x_i)^2 / n, an identity of rational numbers, so the value
    is exact; both sums are the exact ones above (the squares through exact_dot).
    """
    x = np.asarray(x).ravel()
    n = x.size
    s1 = exact_sum(x)
    s2 = exact_dot(x, x)
    return s2 - s1 * s1 / n


def _var_from(ss: Fraction | None, n: int, norm_type: int):
    """Sum of squared deviations over n elements -> variance: divided by n - 1
    (norm_type 0, the default) or by n (norm_type 1); one element gives 0 and no
    elements give None (NaN)."""
    if n == 0 or ss is None:
        return None
    den = n if norm_type == 1 else n - 1
    return Fraction(0) if den == 0 else ss / den


def var(x, dtype: str, norm_type: int = 0):
    """Exact variance of all elements (a Fraction), normalised by N - 1 or N."""
    if dtype not in FLOATS:
        raise ValueError("var is defined here for floating types only")
    x = np.asarray(x)
    if x.size == 0:
        raise ValueError("var of an empty operand")
    _finite_or_raise(x.astype(np.float64))
    return _var_from(_sum_sq_dev(x), x.size, norm_type)


def var_dim(X, dim: int, dtype: str, norm_type: int = 0) -> list:
    """Exact per-column (dim 0) or per-row (dim 1) variances as Fractions (None where
    the count is 0)."""
    if dtype not in FLOATS:
        raise ValueError("var is defined here for floating types only")
    X = np.asarray(X)
    if dim not in (0, 1):
        raise ValueError("dim must be 0 or 1")
    groups = [X[:, j] for j in range(X.shape[1])] if dim == 0 else [X[i, :] for i in range(X.shape[0])]
    out = []
    for g in groups:
        out.append(None if g.size == 0 else _var_from(_sum_sq_dev(g), g.size, norm_type))
    return out


def rel_err(got: float, ref: Fraction, scale: float) -> float:
    """|got - ref| / |ref|, or |got - ref| / scale when ref is 0 (scale = sum |x_i|)."""
    if math.isnan(got):
        return math.inf
    diff = abs(Fraction(got) - ref) if math.isfinite(got) else math.inf
    if ref != 0:
        return float(diff / abs(ref))
    return float(diff) / scale if scale > 0 else float(diff)
