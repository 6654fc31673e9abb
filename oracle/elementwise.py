"""Per-operator, unfused evaluation of a postfix expression (test infrastructure only).

Semantics followed:
  * Section 3 (expression types): eOp / eGlue nodes are element-wise and keep the
    dimensions, and an eGlue needs operands of equal dimensions; Op<.., op_trans>
    swaps the dimensions (the trans() signature shown in Section 3).
  * Section 3 (delayed evaluation): nothing is computed until the whole expression
    is assigned; this oracle then evaluates it the plain way, one operator at a
    time, each into a full temporary.
  * Section 2 (element types): Mat<float>, Mat<double>; u32 / s32 follow the same
    Mat<eT> template, and so do the 16-bit storage types f16 (IEEE binary16) and
    bf16 (bfloat16: binary32's exponent range, 8 significant bits).

Readings where the paper is silent:
  * `%` is the element-wise (Schur) product, as in Armadillo.
  * Floating point: every operator's exact result is rounded once, to nearest-even,
    to the element type; subnormals are kept.  For + - * / and sqrt on binary32
    operands this is computed in binary64 and then rounded to binary32, which is
    exact rounding because 53 >= 2*24 + 2 (double rounding is innocuous).
    exp and log are rounded correctly from a high-precision evaluation.
  * Integers: exact arithmetic reduced mod 2^32 (two's complement for s32);
    abs(INT32_MIN) = INT32_MIN; neg on u32 is 2^32 - x; / exp log sqrt are illegal.
  * A scalar is converted to the element type before use: nearest-even for floats,
    truncation toward zero then mod 2^32 for integers.
  * One dtype per expression; mixing is an error.
  * f16 / bf16 follow the floating rule above with their own rounding: each
    operator's binary64 result (exact for + - * of 16-bit operands, correctly
    rounded for / sqrt exp log) is rounded once more, to nearest-even in the
    16-bit type; 53 >= 2*11 + 2 makes that second rounding innocuous.  bf16 values
    are held in float32 arrays (every bf16 value is a binary32 value).
"""
from __future__ import annotations

import math
from decimal import Decimal, localcontext, InvalidOperation
from fractions import Fraction

import numpy as np

FLOATS = ("f32", "f64", "f16", "bf16")
HALVES = ("f16", "bf16")
INTS = ("u32", "s32")
# element type -> numpy container (bf16 values live in float32 arrays)
NP = {"u32": np.uint32, "s32": np.int32, "f32": np.float32, "f64": np.float64, "f16": np.float16,
      "bf16": np.float32}
BINARY = ("add", "sub", "schur", "div")
UNARY = ("neg", "abs", "exp", "log", "sqrt", "square")
INT_ILLEGAL = ("div", "exp", "log", "sqrt")


class OracleError(Exception):
    """Base class; `kind` is one of 'shape', 'type', 'arity', 'invalid'."""

    def __init__(self, kind, msg):
        super().__init__(msg)
        self.kind = kind


# ---------------------------------------------------------------------------
# Rounding to the 16-bit types
# ---------------------------------------------------------------------------

def round_bf16(x) -> np.ndarray:
    """Round binary64 values to bfloat16, nearest-even, in one step; float32 containers.

    bfloat16 keeps 8 significant bits over binary32's exponent range, so its
    spacing is 2^(e-8) for a value m * 2^e (m in [0.5, 1)) down to the subnormal
    spacing 2^-133.  The value is scaled by a power of two (exact) so that its
    spacing becomes 1, rounded to an integer with ties to even, and scaled back.
    Results of 2^128 or more (the largest finite value plus half its spacing,
    rounded up) become infinite; NaN stays NaN.
    """
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(all="ignore"):
        ax = np.abs(x)
        _, e = np.frexp(ax)
        q = np.maximum(e.astype(np.int64) - 8, -133)
        v = np.ldexp(np.rint(np.ldexp(ax, -q)), q)
        v = np.where(v >= 2.0 ** 128, np.inf, v)
        v = np.where(np.isnan(x), np.nan, np.copysign(v, x))
    return v.astype(np.float32)


def round_to(r64, dtype: str) -> np.ndarray:
    """Round binary64 values to the element type (nearest-even; one rounding)."""
    if dtype == "bf16":
        return round_bf16(r64)
    with np.errstate(all="ignore"):
        return np.asarray(r64, dtype=np.float64).astype(NP[dtype])


def is_bf16(x) -> bool:
    """Every value of a float32 array is a bfloat16 value (its low 16 bits are zero)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    return bool(np.all((b & 0xFFFF) == 0))


# ---------------------------------------------------------------------------
# Scalars
# ---------------------------------------------------------------------------

def scalar_to(s: float, dtype: str):
    """Convert a scalar (a Python float) to the element type."""
    if dtype == "f32":
        return np.float32(s)
    if dtype == "f64":
        return np.float64(s)
    if dtype in HALVES:
        return round_to(np.float64(s), dtype)[()]
    if not math.isfinite(s):
        raise OracleError("invalid", "non-finite scalar for an integer expression")
    v = int(s) & 0xFFFFFFFF          # int() truncates toward zero
    if dtype == "s32" and v >= 1 << 31:
        v -= 1 << 32
    return np.uint32(v) if dtype == "u32" else np.int32(v)


# ---------------------------------------------------------------------------
# Correctly rounded exp / log
# ---------------------------------------------------------------------------

def _round_decimal(v: Decimal, dtype: str):
    """Round a (60-digit) Decimal to binary32/binary64, nearest-even.

    float() of a Decimal is correctly rounded to binary64.  For binary32 a second
    rounding of that binary64 value can only go wrong when the binary64 value is
    exactly a binary32 midpoint; that case is decided with exact arithmetic.
    """
    f = float(v)
    if dtype == "f64":
        return np.float64(f)
    r = np.float32(f)
    if not np.isfinite(r) and math.isfinite(f):
        return r
    # is f exactly halfway between two binary32 neighbours?
    lo = np.float32(f) if float(np.float32(f)) <= f else np.nextafter(np.float32(f), np.float32(-np.inf))
    hi = np.nextafter(lo, np.float32(np.inf))
    if not (np.isfinite(lo) and np.isfinite(hi)):
        return r
    mid = (Fraction(float(lo)) + Fraction(float(hi))) / 2
    if Fraction(f) != mid:
        return r
    exact = Fraction(v)
    if exact > mid:
        return hi
    if exact < mid:
        return lo
    return lo if (int(lo.view(np.uint32)) & 1) == 0 else hi


def _exact_exp(x: float, dtype: str):
    if math.isnan(x):
        return NP[dtype](np.nan)
    if math.isinf(x):
        return NP[dtype](np.inf if x > 0 else 0.0)
    with localcontext() as ctx:
        ctx.prec = 60
        ctx.Emin = -999999
        ctx.Emax = 999999
        v = Decimal(x).exp()
    return _round_decimal(v, dtype)


def _exact_log(x: float, dtype: str):
    if math.isnan(x) or x < 0:
        return NP[dtype](np.nan)
    if x == 0:
        return NP[dtype](-np.inf)
    if math.isinf(x):
        return NP[dtype](np.inf)
    with localcontext() as ctx:
        ctx.prec = 60
        v = Decimal(x).ln()
    return _round_decimal(v, dtype)


def _correctly_rounded(fn_fast, fn_exact, x: np.ndarray, dtype: str) -> np.ndarray:
    """Evaluate a transcendental function correctly rounded to `dtype`.

    Fast path: a wider-precision library evaluation y (binary64 for f32 results,
    x87 extended for f64 results).  If rounding y*(1-m) and y*(1+m) to the target
    gives the same value — m being many times the library's error bound — every
    value in between rounds the same way, so that value is the correctly rounded
    result.  Otherwise the element is recomputed from a 60-digit Decimal.
    """
    if dtype == "f32":
        wide = x.astype(np.float64)
        margin = np.float64(2.0 ** -48)
        target = np.float32
    else:
        wide = x.astype(np.longdouble)
        margin = np.longdouble(2.0 ** -60)
        target = np.float64
    with np.errstate(all="ignore"):
        y = fn_fast(wide)
        a = (y * (1 - margin)).astype(target)
        b = (y * (1 + margin)).astype(target)
        out = y.astype(target)
        ok = (a == b) & ~np.isnan(y)
    bad = np.flatnonzero(~ok.ravel())
    if bad.size:
        flat = out.reshape(-1)
        xs = x.reshape(-1)
        for i in bad:
            flat[i] = fn_exact(float(xs[i]), dtype)
    return out


def exp_rounded(x: np.ndarray, dtype: str) -> np.ndarray:
    """exp(x) correctly rounded to dtype (parity pinned: Decimal brute force, special values)."""
    return _correctly_rounded(np.exp, _exact_exp, np.asarray(x), dtype)


def log_rounded(x: np.ndarray, dtype: str) -> np.ndarray:
    """log(x) correctly rounded to dtype; log(<0) = NaN, log(0) = -inf."""
    return _correctly_rounded(np.log, _exact_log, np.asarray(x), dtype)


# ---------------------------------------------------------------------------
# One operator
# ---------------------------------------------------------------------------

def _float_binary(op, a, b, dtype):
    with np.errstate(all="ignore"):
        a64 = np.asarray(a, dtype=np.float64)
        b64 = np.asarray(b, dtype=np.float64)
        if op == "add":
            r = a64 + b64
        elif op == "sub":
            r = a64 - b64
        elif op == "schur":
            r = a64 * b64
        else:
            r = a64 / b64
        return round_to(r, dtype)


def _float_unary(op, a, dtype):
    t = NP[dtype]
    a = np.asarray(a, dtype=t)
    with np.errstate(all="ignore"):
        if op == "neg":
            return (-a).astype(t)
        if op == "abs":
            return np.abs(a).astype(t)
        if op == "square":
            a64 = a.astype(np.float64)
            return round_to(a64 * a64, dtype)
        if op == "sqrt":
            return round_to(np.sqrt(a.astype(np.float64)), dtype)
        if op in ("exp", "log") and dtype in HALVES:
            # correctly rounded binary64, then rounded to the 16-bit type
            f = exp_rounded if op == "exp" else log_rounded
            return round_to(f(a.astype(np.float64), "f64"), dtype)
        if op == "exp":
            return exp_rounded(a, dtype)
        if op == "log":
            return log_rounded(a, dtype)
    raise OracleError("invalid", op)


_M32 = np.uint64(0xFFFFFFFF)


def _to_u64(a, dtype):
    """Bit pattern of a u32/s32 array, as uint64 in [0, 2^32)."""
    a = np.asarray(a)
    if dtype == "s32":
        return a.astype(np.int32).view(np.uint32).astype(np.uint64)
    return a.astype(np.uint32).astype(np.uint64)


def _from_u64(r, dtype):
    r = (np.asarray(r, dtype=np.uint64) & _M32).astype(np.uint32)
    return r.view(np.int32) if dtype == "s32" else r


def _int_binary(op, a, b, dtype):
    ua, ub = _to_u64(a, dtype), _to_u64(b, dtype)
    with np.errstate(all="ignore"):
        if op == "add":
            r = ua + ub
        elif op == "sub":
            r = ua - ub              # wraps mod 2^64, hence correct mod 2^32
        elif op == "schur":
            r = ua * ub
        else:
            raise OracleError("type", op + " on an integer type")
    return _from_u64(r, dtype)


def _int_unary(op, a, dtype):
    ua = _to_u64(a, dtype)
    with np.errstate(all="ignore"):
        if op == "neg":
            r = np.uint64(0) - ua
        elif op == "square":
            r = ua * ua
        elif op == "abs":
            if dtype == "u32":
                r = ua
            else:
                neg = ua >= np.uint64(1 << 31)
                r = np.where(neg, np.uint64(0) - ua, ua)
        else:
            raise OracleError("type", op + " on an integer type")
    return _from_u64(r, dtype)


# ---------------------------------------------------------------------------
# The whole postfix list
# ---------------------------------------------------------------------------

class _Val:
    """A stack entry: an array of the element type; `scalar` marks a broadcast 1x1 value."""
    __slots__ = ("a", "scalar")

    def __init__(self, a, scalar):
        self.a = a
        self.scalar = scalar

    @property
    def shape(self):
        return None if self.scalar else self.a.shape


def check_dtype(operands, dtype):
    for k, x in enumerate(operands):
        if np.asarray(x).dtype != np.dtype(NP[dtype]):
            raise OracleError("type", f"operand {k} has dtype {np.asarray(x).dtype}, expression is {dtype}")
        if dtype == "bf16" and not is_bf16(x):
            raise OracleError("type", f"operand {k} holds values that are not bfloat16 values")


def evaluate(postfix, operands, scalars, dtype: str) -> np.ndarray:
    """Evaluate a postfix expression one operator at a time.

    postfix   list of tuples, see the `synth` vocabulary
    operands  list of 2-D arrays (logical n_rows x n_cols) of the element type
    scalars   list of Python floats, converted to the element type
    returns   2-D array of the element type, or a 1x1 array if the expression is scalar-only
    Raises OracleError for arity, shape and dtype errors.
    """
    check_dtype(operands, dtype)
    is_int = dtype in INTS
    st: list[_Val] = []
    for item in postfix:
        op = item[0]
        if op == "load":
            k = item[1]
            if not 0 <= k < len(operands):
                raise OracleError("invalid", f"operand slot {k} out of range")
            st.append(_Val(np.asarray(operands[k]), False))
        elif op == "scalar":
            k = item[1]
            if not 0 <= k < len(scalars):
                raise OracleError("invalid", f"scalar slot {k} out of range")
            st.append(_Val(np.asarray(scalar_to(scalars[k], dtype)), True))
        elif op in BINARY:
            if len(st) < 2:
                raise OracleError("arity", f"{op} needs two operands")
            b = st.pop()
            a = st.pop()
            if not a.scalar and not b.scalar and a.shape != b.shape:
                raise OracleError("shape", f"{op}: {a.shape} vs {b.shape}")
            if is_int:
                if op in INT_ILLEGAL:
                    raise OracleError("type", op + " on an integer type")
                r = _int_binary(op, a.a, b.a, dtype)
            else:
                r = _float_binary(op, a.a, b.a, dtype)
            st.append(_Val(np.asarray(r), a.scalar and b.scalar))
        elif op in UNARY:
            if not st:
                raise OracleError("arity", f"{op} needs an operand")
            a = st.pop()
            if is_int:
                if op in INT_ILLEGAL:
                    raise OracleError("type", op + " on an integer type")
                r = _int_unary(op, a.a, dtype)
            else:
                r = _float_unary(op, a.a, dtype)
            st.append(_Val(np.asarray(r), a.scalar))
        elif op == "trans":
            if not st:
                raise OracleError("arity", "trans needs an operand")
            a = st.pop()
            st.append(_Val(a.a if a.scalar else np.ascontiguousarray(a.a.T), a.scalar))
        else:
            raise OracleError("invalid", f"unknown op {op!r}")
    if len(st) != 1:
        raise OracleError("arity", f"expression leaves {len(st)} values on the stack")
    v = st[0]
    if v.scalar:
        return np.asarray(v.a).reshape(1, 1)
    return np.asarray(v.a)


def out_shape(postfix, slot_shapes):
    """Shape inference alone: (n_rows, n_cols) of the result, or None for a scalar-only tree."""
    st = []
    for item in postfix:
        op = item[0]
        if op == "load":
            st.append(tuple(slot_shapes[item[1]]))
        elif op == "scalar":
            st.append(None)
        elif op in BINARY:
            if len(st) < 2:
                raise OracleError("arity", op)
            b, a = st.pop(), st.pop()
            if a is not None and b is not None and a != b:
                raise OracleError("shape", f"{op}: {a} vs {b}")
            st.append(a if a is not None else b)
        elif op in UNARY:
            if not st:
                raise OracleError("arity", op)
        elif op == "trans":
            if not st:
                raise OracleError("arity", op)
            a = st.pop()
            st.append(None if a is None else (a[1], a[0]))
        else:
            raise OracleError("invalid", op)
    if len(st) != 1:
        raise OracleError("arity", "stack")
    return st[0]


def evaluate_at(postfix, operands, scalars, dtype: str, rows, cols) -> np.ndarray:
    """Values of the expression at the given output coordinates only.

    Used where the full result is too large for the oracle: every leaf is read at
    the coordinate its index map gives (an odd number of trans() above a leaf swaps
    row and column), and the operators are then applied one at a time to those
    1-D samples exactly as `evaluate` applies them to whole temporaries.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    # parity of each postfix position: number of trans() ancestors mod 2
    n = len(postfix)
    parent_flip = [0] * n
    # walk the postfix list backwards with an explicit stack of pending parities
    pend = [0]
    for i in range(n - 1, -1, -1):
        op = postfix[i][0]
        p = pend.pop()
        parent_flip[i] = p
        if op in BINARY:
            pend.extend([p, p])
        elif op in UNARY:
            pend.append(p)
        elif op == "trans":
            pend.append(p ^ 1)
    sampled = []
    remap = []
    for i, item in enumerate(postfix):
        if item[0] == "load":
            x = np.asarray(operands[item[1]])
            if parent_flip[i]:
                vals = x[cols, rows]
            else:
                vals = x[rows, cols]
            sampled.append(vals.reshape(-1, 1))
            remap.append(("load", len(sampled) - 1))
        elif item[0] == "trans":
            continue                  # index map already applied at the leaves
        else:
            remap.append(item)
    return evaluate(remap, sampled, scalars, dtype).reshape(-1)
