"""The oracle's 16-bit element types (f16, bf16) pinned to the rounding definition.

Rounding is checked against a brute-force search over every finite value of the
type (exact rationals, ties to the even significand), an implementation that
shares nothing with the oracle's scaling method; worked examples fix the
per-operator semantics."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from oracle import reduce as rd


def _all_finite(dtype):
    """Sorted non-negative finite values of the type and, for each, whether its significand is even."""
    bits = np.arange(0, 1 << 16, dtype=np.uint32)
    with np.errstate(invalid="ignore"):
        if dtype == "f16":
            v = bits.astype(np.uint16).view(np.float16).astype(np.float64)
        else:
            v = (bits << 16).view(np.float32).astype(np.float64)
    keep = np.isfinite(v) & (v >= 0) & ~np.signbit(v)
    vals, b = v[keep], bits[keep]
    order = np.argsort(vals, kind="stable")
    return vals[order], (b[order] & 1) == 0


def _brute_round(x: float, vals, even, top_half_ulp: Fraction):
    """Nearest value of the sorted table (ties to the even pattern); overflow -> inf."""
    ax = abs(x)
    largest = Fraction(float(vals[-1]))
    if Fraction(ax) >= largest + top_half_ulp:
        return math.copysign(math.inf, x)
    i = int(np.searchsorted(vals, ax, side="right")) - 1
    lo = Fraction(float(vals[i]))
    if i + 1 == len(vals):
        return math.copysign(float(vals[i]), x)
    hi = Fraction(float(vals[i + 1]))
    d_lo, d_hi = Fraction(ax) - lo, hi - Fraction(ax)
    if d_lo < d_hi or (d_lo == d_hi and even[i]):
        r = float(vals[i])
    else:
        r = float(vals[i + 1])
    return math.copysign(r, x)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_rounding_matches_brute_force(dtype):
    vals, even = _all_finite(dtype)
    top_half_ulp = Fraction(2) ** (4 if dtype == "f16" else 119)   # half the spacing at the largest finite value
    g = np.random.default_rng(11)
    lo_e, hi_e = (-27, 17) if dtype == "f16" else (-136, 129)
    xs = [float(g.uniform(1, 2) * 2.0 ** int(g.integers(lo_e, hi_e)) * (1 if g.random() < 0.5 else -1))
          for _ in range(3000)]
    # exact midpoints between neighbours, and their one-ulp (binary64) neighbours
    for i in g.integers(0, len(vals) - 1, 400):
        m = (float(vals[i]) + float(vals[i + 1])) / 2
        xs += [m, math.nextafter(m, 0), math.nextafter(m, math.inf)]
    got = ew.round_to(np.array(xs), dtype).astype(np.float64)
    for x, r in zip(xs, got):
        want = _brute_round(x, vals, even, top_half_ulp)
        assert r == want or (math.isnan(r) and math.isnan(want)), (dtype, x.hex(), float(r), want)


def test_bf16_values_round_to_themselves():
    bits = (np.arange(0, 1 << 16, dtype=np.uint32) << 16).view(np.float32)
    with np.errstate(invalid="ignore"):
        r = ew.round_bf16(bits.astype(np.float64))
    same = (r.view(np.uint32) == bits.view(np.uint32)) | (np.isnan(r) & np.isnan(bits))
    assert same.all()


def test_worked_examples():
    ev = ew.evaluate
    one = lambda dt: [np.full((1, 1), 1.0, ew.NP[dt])]
    # f16: spacing 2^-10 at 1; 1 + 2^-11 is a tie -> 1 (even); 1 + 2^-10 + 2^-11 -> 1 + 2^-9
    assert ev([("load", 0), ("scalar", 0), ("add",)], one("f16"), [2.0 ** -11], "f16")[0, 0] == 1.0
    a = [np.full((1, 1), 1 + 2.0 ** -10, np.float16)]
    assert ev([("load", 0), ("scalar", 0), ("add",)], a, [2.0 ** -11], "f16")[0, 0] == 1 + 2.0 ** -9
    # f16 overflow: 65504 + 16 is the tie between the largest value and 2^16 -> inf
    big = [np.full((1, 1), 65504.0, np.float16)]
    assert ev([("load", 0), ("scalar", 0), ("add",)], big, [16.0], "f16")[0, 0] == np.inf
    assert ev([("load", 0), ("scalar", 0), ("add",)], big, [15.0], "f16")[0, 0] == 65504.0
    # bf16: spacing 2^-7 at 1; 1 + 2^-8 -> 1; (1 + 2^-7) + 2^-8 -> 1 + 2^-6
    assert ev([("load", 0), ("scalar", 0), ("add",)], one("bf16"), [2.0 ** -8], "bf16")[0, 0] == 1.0
    b = [np.full((1, 1), 1 + 2.0 ** -7, np.float32)]
    assert ev([("load", 0), ("scalar", 0), ("add",)], b, [2.0 ** -8], "bf16")[0, 0] == 1 + 2.0 ** -6
    # a scalar is rounded to the type first: 0.1 -> the nearest value of each type
    assert float(ew.scalar_to(0.1, "f16")) == 1638 * 2.0 ** -14
    assert float(ew.scalar_to(0.1, "bf16")) == 205 * 2.0 ** -11
    # exp(1) = 2.71828...: f16 spacing 2^-9 at 2 gives 1392 * 2^-9, bf16 spacing 2^-6 gives 174 * 2^-6
    assert ev([("load", 0), ("exp",)], one("f16"), [], "f16")[0, 0] == 1392 * 2.0 ** -9
    assert ev([("load", 0), ("exp",)], one("bf16"), [], "bf16")[0, 0] == 174 * 2.0 ** -6
    # division and sqrt: 1/3 and sqrt(2) to the nearest value of each type
    three = [np.full((1, 1), 3.0, np.float16)]
    assert ev([("scalar", 0), ("load", 0), ("div",)], three, [1.0], "f16")[0, 0] == 1365 * 2.0 ** -12
    two = [np.full((1, 1), 2.0, np.float32)]
    assert ev([("load", 0), ("sqrt",)], two, [], "bf16")[0, 0] == 181 * 2.0 ** -7


def test_bf16_operands_are_checked():
    with pytest.raises(ew.OracleError):
        ew.evaluate([("load", 0)], [np.full((1, 1), 0.1, np.float32)], [], "bf16")


def test_exact_reductions_rounded_to_the_type():
    # 2049 ones: the exact sum 2049 is a tie in f16 (spacing 2 in [2048, 4096)) -> 2048 (even)
    x = np.ones((2049, 1), np.float16)
    assert rd.round_exact(rd.accu(x, "f16"), "f16") == 2048.0
    x[0] = 3.0                                                       # exact sum 2051: a tie -> 2052
    assert rd.round_exact(rd.accu(x, "f16"), "f16") == 2052.0
    y = np.full((257, 1), 1.0, np.float32)
    assert rd.round_exact(rd.accu(y, "bf16"), "bf16") == 256.0         # 257 is a tie (spacing 2) -> 256
    assert rd.round_exact(rd.dot(y, y, "bf16"), "bf16") == 256.0


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_synthetic_inputs_of_the_type(dtype):
    g = synth.rng_for(5)
    a = synth.uniform(g, (64, 33), dtype)
    assert a.dtype == ew.NP[dtype] and np.all(np.abs(a) <= 1)
    if dtype == "bf16":
        assert ew.is_bf16(a)
    spec = synth.random_tree(g, 3, 3, 5, 6, dtype)
    ops = synth.operands_for(spec, g)
    assert all(o.dtype == ew.NP[dtype] for o in ops)
    assert ew.evaluate(spec.postfix, ops, spec.scalars, dtype).dtype == ew.NP[dtype]
