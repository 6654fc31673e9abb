"""Pins for the reduction oracle (CPU only): Fraction brute force, closed forms,
overflow / underflow cases and integer wrap-around."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import reduce as rd


def _wide_f32(rng, n):
    e = rng.uniform(-140, 120, n)
    return (np.sign(rng.uniform(-1, 1, n)) * np.exp2(e)).astype(np.float32)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_exact_sum_against_fraction_brute_force(dtype):
    rng = np.random.default_rng(10)
    for n in (0, 1, 2, 7, 100, 1000):
        x = _wide_f32(rng, n).astype(np.float64 if dtype == "f64" else np.float32)
        if dtype == "f64":
            x = x * np.exp2(rng.uniform(-900, 900, n))
        want = sum((Fraction(float(v)) for v in x), Fraction(0))
        assert rd.exact_sum(x) == want
        assert rd.accu(x, dtype) == want


def test_exact_sum_closed_forms():
    assert rd.exact_sum(np.ones(1 << 20, np.float32)) == 1 << 20
    x = np.concatenate([[np.float32(2 ** 24)], np.ones(1 << 20, np.float32)])
    assert rd.exact_sum(x) == 2 ** 24 + 2 ** 20
    naive = np.float32(0)
    for v in x[:5]:
        naive = np.float32(naive + v)
    assert naive == np.float32(2 ** 24)          # plain fp32 summation loses the ones
    assert rd.exact_sum(np.array([1e8, 1, -1e8], np.float32)) == 1
    # a Gaussian-integer closed form: sum_{k<n} k
    n = 100_000
    assert rd.exact_sum(np.arange(n, dtype=np.float64)) == n * (n - 1) // 2


def test_exact_sum_chunk_boundaries(monkeypatch):
    # several summation passes: the pass boundaries must not lose anything
    monkeypatch.setattr(rd, "CHUNK", 1000)
    rng = np.random.default_rng(14)
    x = _wide_f32(rng, 12345)
    y = _wide_f32(rng, 12345)
    assert rd.exact_sum(x) == sum((Fraction(float(v)) for v in x), Fraction(0))
    assert rd.exact_dot(x.astype(np.float64), y.astype(np.float64)) == \
        sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    n = 100_003
    assert rd.exact_sum(np.full(n, 0.5, dtype=np.float32)) == Fraction(n, 2)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_exact_dot_against_fraction(dtype):
    rng = np.random.default_rng(11)
    t = np.float32 if dtype == "f32" else np.float64
    for n in (0, 1, 5, 300):
        x = rng.uniform(-1, 1, n).astype(t) * t(2.0) ** rng.integers(-60, 60, n).astype(t)
        y = rng.uniform(-1, 1, n).astype(t) * t(2.0) ** rng.integers(-60, 60, n).astype(t)
        want = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
        assert rd.exact_dot(x, y) == want


def test_norm_closed_forms():
    # squares overflow (2^200) or underflow (2^-200) binary32, the norm itself does not
    big = np.array([3 * 2.0 ** 100, 4 * 2.0 ** 100], np.float32)
    small = np.array([3 * 2.0 ** -100, 4 * 2.0 ** -100], np.float32)
    assert rd.norm(big, "f32") == 5 * 2.0 ** 100
    assert rd.norm(small, "f32") == 5 * 2.0 ** -100
    assert rd.norm(np.array([3.0, 4.0], np.float32), "f32") == 5.0
    assert rd.norm(np.zeros(5, np.float32), "f32") == 0.0
    rng = np.random.default_rng(12)
    v = rng.uniform(-1, 1, 4000).astype(np.float32)
    n2 = Fraction(rd.norm(v, "f32")) ** 2
    d = rd.exact_dot(v, v)
    assert abs(n2 - d) / d < Fraction(1, 10 ** 15)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sum_dim_against_per_column_fractions(dtype):
    rng = np.random.default_rng(13)
    t = np.float32 if dtype == "f32" else np.float64
    X = (rng.uniform(-1, 1, (9, 6)) * np.exp2(rng.integers(-30, 30, (9, 6)))).astype(t)
    s0 = rd.sum_dim(X, 0, dtype)
    s1 = rd.sum_dim(X, 1, dtype)
    assert len(s0) == 6 and len(s1) == 9
    for j in range(6):
        assert s0[j] == sum((Fraction(float(v)) for v in X[:, j]), Fraction(0))
    for i in range(9):
        assert s1[i] == sum((Fraction(float(v)) for v in X[i, :]), Fraction(0))
    # invariant: summing either set of partial sums gives accu
    assert sum(s0, Fraction(0)) == sum(s1, Fraction(0)) == rd.accu(X, dtype)
    # sum(trans(X), 0) == trans(sum(X, 1))
    assert rd.sum_dim(np.ascontiguousarray(X.T), 0, dtype) == s1
    assert rd.sum_dim(np.zeros((0, 4), t), 0, dtype) == [0, 0, 0, 0]


def test_integer_accu_closed_form_and_wrap():
    n = 100_000
    u = np.arange(n, dtype=np.uint32)
    assert rd.accu(u, "u32") == (n * (n - 1) // 2) % 2 ** 32
    s = synth.uniform_int(synth.rng_for(50), (50, 40), "s32", -(1 << 31), 1 << 31)
    want = sum(int(v) for v in s.ravel()) % 2 ** 32
    want = want - 2 ** 32 if want >= 2 ** 31 else want
    assert rd.accu(s, "s32") == want
    cols = rd.sum_dim(s, 0, "s32")
    for j in range(40):
        w = sum(int(v) for v in s[:, j]) % 2 ** 32
        assert cols[j] == (w - 2 ** 32 if w >= 2 ** 31 else w)


def test_rel_err():
    assert rd.rel_err(1.0, Fraction(1), 1.0) == 0
    assert rd.rel_err(1.5, Fraction(1), 1.0) == 0.5
    assert rd.rel_err(1e-3, Fraction(0), 10.0) == pytest.approx(1e-4)
    assert rd.rel_err(float("nan"), Fraction(1), 1.0) == math.inf
