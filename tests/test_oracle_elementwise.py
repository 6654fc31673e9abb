"""Pins for the element-wise oracle (CPU only).

Each check compares the oracle with something other than itself: exact rational
arithmetic plus IEEE rounding written from the definition (tests/exact.py), a
pure-Python big-integer walker for u32/s32, 80-digit Decimal for exp, and
algebraic identities that hold exactly.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from tests import exact

F32 = np.float32


def _edge_f32(rng, n):
    """Random binary32 values spanning normal, subnormal, tiny and huge magnitudes and zeros."""
    bits = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    extra = np.array([0.0, -0.0, 1.0, -1.0, 2.5, 1e-45, -1e-45, 1.1754944e-38, 3.4028235e38,
                      -3.4028235e38, 0.1, 1 / 3], dtype=np.float32)
    return np.concatenate([extra, x, rng.uniform(-1, 1, n).astype(np.float32)])


@pytest.mark.parametrize("op", ["add", "sub", "schur", "div"])
def test_f32_binary_ops_are_exactly_rounded(op):
    rng = np.random.default_rng(1)
    a = _edge_f32(rng, 1500)
    b = _edge_f32(rng, 1500)[: a.size]
    rng.shuffle(b)
    got = ew.evaluate([("load", 0), ("load", 1), (op,)], [a.reshape(-1, 1), b.reshape(-1, 1)], [], "f32").ravel()
    for i in range(a.size):
        if op == "div" and b[i] == 0:
            continue
        want = exact.binop(op, a[i], b[i], "f32")
        g = got[i]
        assert (np.isnan(g) and np.isnan(want)) or (g == want and math.copysign(1, g) == math.copysign(1, want)), \
            (op, a[i], b[i], g, want)


@pytest.mark.parametrize("op", ["add", "sub", "schur", "div"])
def test_f64_binary_ops_are_exactly_rounded(op):
    rng = np.random.default_rng(2)
    bits = rng.integers(0, 1 << 63, size=600, dtype=np.uint64) | (rng.integers(0, 2, size=600, dtype=np.uint64) << np.uint64(63))
    a = bits.view(np.float64)
    a = a[np.isfinite(a)]
    a = np.concatenate([a, rng.uniform(-1, 1, 400), [5e-324, -5e-324, 0.0, -0.0]])
    b = a.copy()
    rng.shuffle(b)
    got = ew.evaluate([("load", 0), ("load", 1), (op,)], [a.reshape(-1, 1), b.reshape(-1, 1)], [], "f64").ravel()
    for i in range(a.size):
        if op == "div" and b[i] == 0:
            continue
        want = exact.binop(op, a[i], b[i], "f64")
        assert got[i] == want or (np.isnan(got[i]) and np.isnan(want)), (op, a[i], b[i])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sqrt_and_square_exactly_rounded(dtype):
    rng = np.random.default_rng(3)
    t = np.float32 if dtype == "f32" else np.float64
    with np.errstate(over="ignore"):
        x = np.abs(np.concatenate([rng.uniform(0, 4, 300), np.exp(rng.uniform(-200, 200, 300)), [0.0, 2.0, 1e-45]])).astype(t)
    x = x[np.isfinite(x)]
    sq = ew.evaluate([("load", 0), ("sqrt",)], [x.reshape(-1, 1)], [], dtype).ravel()
    sqr = ew.evaluate([("load", 0), ("square",)], [x.reshape(-1, 1)], [], dtype).ravel()
    for i in range(x.size):
        assert sq[i] == exact.exact_sqrt_rounded(Fraction(float(x[i])), dtype)
        assert sqr[i] == exact.round_fraction(Fraction(float(x[i])) ** 2, dtype)


def test_exp_f32_correctly_rounded_against_decimal():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(-1, 1, 1500), rng.uniform(-104, 89, 1500),
                        [0.0, -0.0, 88.72283, 88.72284, -87.33654, -103.27893, -103.97208, -104.0, 1e-8, -1e-8]]
                       ).astype(np.float32)
    got = ew.exp_rounded(x, "f32")
    for i in range(x.size):
        want = exact.exp_rounded(float(x[i]), "f32")
        assert got[i] == want, (x[i], got[i], want)


def test_exp_f64_correctly_rounded_against_decimal():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(-1, 1, 800), rng.uniform(-745, 709.7, 800), [0.0, 709.78, -744.5, 1e-17]])
    got = ew.exp_rounded(x, "f64")
    for i in range(x.size):
        want = exact.exp_rounded(float(x[i]), "f64")
        assert got[i] == want, (x[i], got[i], want)


def test_exp_special_values_and_monotone():
    x = np.array([np.nan, np.inf, -np.inf, 0.0, 89.0, -110.0], dtype=np.float32)
    y = ew.exp_rounded(x, "f32")
    assert np.isnan(y[0]) and y[1] == np.inf and y[2] == 0 and y[3] == 1 and y[4] == np.inf and y[5] == 0
    xs = np.sort(np.random.default_rng(6).uniform(-90, 89, 20000).astype(np.float32))
    ys = ew.exp_rounded(xs, "f32")
    assert np.all(ys[1:] >= ys[:-1])


def test_log_matches_decimal_and_specials():
    rng = np.random.default_rng(7)
    x = np.exp(rng.uniform(-80, 80, 500)).astype(np.float32)
    got = ew.log_rounded(x, "f32")
    from decimal import Decimal, localcontext
    for i in range(x.size):
        with localcontext() as ctx:
            ctx.prec = 80
            want = exact.round_fraction(Fraction(Decimal(float(x[i])).ln()), "f32")
        assert got[i] == want
    s = ew.log_rounded(np.array([0.0, -1.0, 1.0, np.inf], dtype=np.float32), "f32")
    assert s[0] == -np.inf and np.isnan(s[1]) and s[2] == 0 and s[3] == np.inf


def _decimal_log_rounded(x: float, dtype: str):
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 80
        return exact.round_fraction(Fraction(Decimal(x).ln()), dtype)


def test_log_f64_correctly_rounded_against_decimal():
    """The binary64 branch (extended-precision fast path, Decimal fallback) against an
    80-digit Decimal logarithm rounded by the IEEE definition: wide magnitudes,
    subnormals, values next to 1 (where log is tiny and its rounding hardest) and
    exact powers of two."""
    rng = np.random.default_rng(8)
    x = np.concatenate([np.exp(rng.uniform(-700, 700, 600)), rng.uniform(0.5, 2.0, 300),
                        1.0 + np.arange(1, 40) * 2.0 ** -52, 1.0 - np.arange(1, 40) * 2.0 ** -53,
                        2.0 ** np.arange(-1074, 1024, 37).astype(np.float64),
                        [5e-324, 1e-310, 2.2250738585072014e-308, 1.7976931348623157e308, 0.1, 10.0, 3.0]])
    got = ew.log_rounded(x, "f64")
    for i in range(x.size):
        want = _decimal_log_rounded(float(x[i]), "f64")
        assert got[i] == want, (float(x[i]), float(got[i]), float(want))
    s = ew.log_rounded(np.array([0.0, -0.0, -1.0, 1.0, np.inf, np.nan]), "f64")
    assert s[0] == -np.inf and s[1] == -np.inf and np.isnan(s[2]) and s[3] == 0 and s[4] == np.inf
    assert np.isnan(s[5])


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_log_of_16bit_values_against_decimal(dtype):
    """16-bit log (binary64 log correctly rounded, then rounded to the type) equals the
    80-digit Decimal logarithm rounded straight to the type by a brute-force search
    over its finite values: every positive finite f16 value, a bf16 sample."""
    from tests.test_oracle_halves import _all_finite, _brute_round
    vals, even = _all_finite(dtype)
    top_half_ulp = Fraction(2) ** (4 if dtype == "f16" else 119)
    pos = vals[vals > 0]
    if dtype == "bf16":
        pos = pos[np.random.default_rng(9).choice(pos.size, 3000, replace=False)]
    x = pos.astype(np.float16) if dtype == "f16" else pos.astype(np.float32)
    got = ew.evaluate([("load", 0), ("log",)], [x.reshape(-1, 1)], [], dtype).ravel()
    from decimal import Decimal, localcontext
    for i in range(x.size):
        with localcontext() as ctx:
            ctx.prec = 80
            q = Decimal(float(x[i])).ln()
        # the 80-digit value lies between the binary64 neighbours of float(q); when
        # both round to the same 16-bit value, so does the 80-digit value
        f = float(q)
        want = _brute_round(f, vals, even, top_half_ulp)
        assert _brute_round(math.nextafter(f, -math.inf), vals, even, top_half_ulp) == want
        assert _brute_round(math.nextafter(f, math.inf), vals, even, top_half_ulp) == want
        assert float(got[i]) == want, (float(x[i]), float(got[i]), want)


def _py_int_eval(postfix, ops, scalars, dtype, i, j):
    """Pure-Python big-integer evaluation of one output element, reduced mod 2^32 per op."""
    M = 1 << 32

    def norm(v):
        v %= M
        if dtype == "s32" and v >= 1 << 31:
            v -= M
        return v

    par = [0] * len(postfix)
    pend = [0]
    for k in range(len(postfix) - 1, -1, -1):
        p = pend.pop()
        par[k] = p
        o = postfix[k][0]
        if o in ("add", "sub", "schur"):
            pend += [p, p]
        elif o in ("neg", "abs", "square"):
            pend.append(p)
        elif o == "trans":
            pend.append(p ^ 1)
    st = []
    for k, it in enumerate(postfix):
        o = it[0]
        if o == "load":
            x = ops[it[1]]
            st.append(int(x[j, i]) if par[k] else int(x[i, j]))
        elif o == "scalar":
            st.append(norm(int(scalars[it[1]])))
        elif o in ("add", "sub", "schur"):
            b, a = st.pop(), st.pop()
            st.append(norm(a + b if o == "add" else a - b if o == "sub" else a * b))
        elif o == "neg":
            st.append(norm(-st.pop()))
        elif o == "square":
            a = st.pop()
            st.append(norm(a * a))
        elif o == "abs":
            a = st.pop()
            st.append(norm(abs(a)))
        elif o == "trans":
            pass
    return st[0]


@pytest.mark.parametrize("dtype", ["u32", "s32"])
def test_integer_trees_against_big_int_walker(dtype):
    g = synth.rng_for(99, 1 if dtype == "u32" else 2)
    for trial in range(40):
        r, c = int(g.integers(1, 7)), int(g.integers(1, 7))
        spec = synth.random_tree(g, int(g.integers(1, 7)), int(g.integers(2, 6)), r, c, dtype)
        lo, hi = (0, 1 << 32) if dtype == "u32" else (-(1 << 31), 1 << 31)
        ops = [synth.uniform_int(g, s, dtype, lo, hi) for s in spec.slot_shapes]
        got = ew.evaluate(spec.postfix, ops, spec.scalars, dtype)
        assert got.shape == (r, c)
        for i in range(r):
            for j in range(c):
                assert int(got[i, j]) == _py_int_eval(spec.postfix, ops, spec.scalars, dtype, i, j), spec.postfix


def test_integer_wrap_cases():
    u = np.array([[0, 1, 0xFFFFFFFF, 65535]], dtype=np.uint32)
    assert list(ew.evaluate([("load", 0), ("neg",)], [u], [], "u32").ravel()) == [0, 0xFFFFFFFF, 1, 2 ** 32 - 65535]
    s = np.array([[-(2 ** 31), -1, 2 ** 31 - 1]], dtype=np.int32)
    assert list(ew.evaluate([("load", 0), ("abs",)], [s], [], "s32").ravel()) == [-(2 ** 31), 1, 2 ** 31 - 1]
    # (A + B) % C on the u32 range of the integer workload wraps: (2^17 - 2) * (2^16 - 1) > 2^32
    a = np.array([[65535]], dtype=np.uint32)
    r = ew.evaluate([("load", 0), ("load", 0), ("add",), ("load", 0), ("schur",)], [a], [], "u32")
    assert int(r[0, 0]) == ((65535 + 65535) * 65535) % 2 ** 32
    # scalar conversion truncates toward zero: 2.5 -> 2, -2.5 -> -2
    assert int(ew.evaluate([("scalar", 0), ("load", 0), ("schur",)], [s], [2.5], "s32")[0, 1]) == -2
    assert int(ew.evaluate([("scalar", 0), ("load", 0), ("schur",)], [s], [-2.5], "s32")[0, 1]) == 2


def _frac_eval(postfix, ops, scalars, dtype, i, j):
    """Scalar tree walker over exact rationals, rounding after every operator (floats)."""
    par = [0] * len(postfix)
    pend = [0]
    for k in range(len(postfix) - 1, -1, -1):
        p = pend.pop()
        par[k] = p
        o = postfix[k][0]
        if o in ("add", "sub", "schur", "div"):
            pend += [p, p]
        elif o in ("neg", "abs", "square", "sqrt", "exp", "log"):
            pend.append(p)
        elif o == "trans":
            pend.append(p ^ 1)
    st = []
    t = exact.FMT[dtype][3]
    for k, it in enumerate(postfix):
        o = it[0]
        if o == "load":
            x = ops[it[1]]
            st.append(t(x[j, i]) if par[k] else t(x[i, j]))
        elif o == "scalar":
            st.append(t(scalars[it[1]]))
        elif o in ("add", "sub", "schur", "div"):
            b, a = st.pop(), st.pop()
            st.append(exact.binop(o, a, b, dtype))
        elif o == "neg":
            st.append(t(-st.pop()))
        elif o == "abs":
            st.append(t(abs(st.pop())))
        elif o == "square":
            a = st.pop()
            st.append(exact.binop("schur", a, a, dtype))
        elif o == "sqrt":
            st.append(exact.exact_sqrt_rounded(Fraction(float(st.pop())), dtype))
        elif o == "exp":
            st.append(exact.exp_rounded(float(st.pop()), dtype))
    return st[0]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_float_trees_bitwise_against_rational_walker(dtype):
    g = synth.rng_for(98, 1 if dtype == "f32" else 2)
    for trial in range(30):
        r, c = int(g.integers(1, 6)), int(g.integers(1, 6))
        spec = synth.random_tree(g, int(g.integers(1, 7)), int(g.integers(2, 6)), r, c, dtype)
        ops = synth.operands_for(spec, g)
        got = ew.evaluate(spec.postfix, ops, spec.scalars, dtype)
        for i in range(r):
            for j in range(c):
                want = _frac_eval(spec.postfix, ops, spec.scalars, dtype, i, j)
                assert got[i, j] == want, (spec.postfix, i, j, got[i, j], want)


def test_contraction_detector():
    """2.5*x + y rounded per operator differs from the singly rounded fused value."""
    x = F32(0.1)
    p = exact.binop("schur", F32(2.5), x, "f32")
    y = F32(-p) + F32(2.0 ** -30)   # y = -rn(2.5x) + tiny, exactly representable
    y = F32(y)
    per_op = exact.binop("add", p, y, "f32")
    fused = exact.round_fraction(Fraction(2.5) * Fraction(float(x)) + Fraction(float(y)), "f32")
    assert per_op != fused
    got = ew.evaluate([("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("add",)],
                      [np.array([[x]]), np.array([[y]])], [2.5], "f32")
    assert got[0, 0] == per_op


def test_transpose_and_identities():
    g = synth.rng_for(97)
    A = synth.uniform(g, (5, 3), "f32")
    tt = ew.evaluate([("load", 0), ("trans",), ("trans",)], [A], [], "f32")
    assert np.array_equal(tt, A)
    t1 = ew.evaluate([("load", 0), ("trans",)], [A], [], "f32")
    assert t1.shape == (3, 5)
    for i in range(3):
        for j in range(5):
            assert t1[i, j] == A[j, i]
    two_a = ew.evaluate([("scalar", 0), ("load", 0), ("schur",)], [A], [2.0], "f32")
    a_plus_a = ew.evaluate([("load", 0), ("load", 0), ("add",)], [A], [], "f32")
    assert np.array_equal(two_a, a_plus_a)
    assert np.all(ew.evaluate([("load", 0), ("load", 0), ("sub",)], [A], [], "f32") == 0)
    assert np.array_equal(ew.evaluate([("load", 0), ("neg",), ("abs",)], [A], [], "f32"),
                          ew.evaluate([("load", 0), ("abs",)], [A], [], "f32"))
    z = ew.evaluate([("load", 0), ("abs",)], [np.array([[-0.0]], dtype=np.float32)], [], "f32")
    assert math.copysign(1, z[0, 0]) > 0


def test_errors():
    A = np.zeros((2, 3), np.float32)
    B = np.zeros((3, 2), np.float32)
    with pytest.raises(ew.OracleError) as e:
        ew.evaluate([("load", 0), ("load", 1), ("add",)], [A, B], [], "f32")
    assert e.value.kind == "shape"
    assert ew.evaluate([("load", 0), ("load", 1), ("trans",), ("add",)], [A, B], [], "f32").shape == (2, 3)
    with pytest.raises(ew.OracleError) as e:
        ew.evaluate([("load", 0), ("add",)], [A], [], "f32")
    assert e.value.kind == "arity"
    with pytest.raises(ew.OracleError) as e:
        ew.evaluate([("load", 0), ("exp",)], [np.zeros((1, 1), np.uint32)], [], "u32")
    assert e.value.kind == "type"
    with pytest.raises(ew.OracleError) as e:
        ew.evaluate([("load", 0), ("load", 1), ("add",)], [A, np.zeros((2, 3), np.float64)], [], "f32")
    assert e.value.kind == "type"
    assert ew.out_shape([("load", 0), ("trans",), ("scalar", 0), ("add",)], [(2, 3)]) == (3, 2)


def test_evaluate_at_matches_full_evaluation():
    g = synth.rng_for(96)
    for trial in range(20):
        r, c = int(g.integers(1, 9)), int(g.integers(1, 9))
        spec = synth.random_tree(g, int(g.integers(1, 7)), int(g.integers(2, 6)), r, c, "f32")
        ops = synth.operands_for(spec, g)
        full = ew.evaluate(spec.postfix, ops, spec.scalars, "f32")
        rows = g.integers(0, r, 17)
        cols = g.integers(0, c, 17)
        part = ew.evaluate_at(spec.postfix, ops, spec.scalars, "f32", rows, cols)
        assert np.array_equal(part, full[rows, cols])


def test_workload_expressions_small():
    """The 2-D workload expressions on a small case, element by element against the rational walker."""
    A, B, C, D = synth.matrix_inputs(n_rows=7, n_cols=5)
    z = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",),
         ("load", 3), ("trans",), ("sub",)]
    w = [("load", 0), ("exp",), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]
    Z = ew.evaluate(z, [A, B, C, D], [2.0], "f32")
    W = ew.evaluate(w, [A, B], [1.0], "f32")
    for i in range(7):
        for j in range(5):
            assert Z[i, j] == _frac_eval(z, [A, B, C, D], [2.0], "f32", i, j)
            assert W[i, j] == _frac_eval(w, [A, B], [1.0], "f32", i, j)
