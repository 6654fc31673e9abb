"""Pins for the oracle's statistics (mean along a dimension, variance): brute force
over Fractions on small inputs, closed forms, invariances, and numpy's float64
results on well-conditioned data."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import reduce as rd


def _brute_var(x, norm_type=0):
    """sum (x_i - mu)^2 / (n - 1) (or / n), every step a Fraction."""
    v = [Fraction(float(t)) for t in np.asarray(x).ravel()]
    n = len(v)
    mu = sum(v, Fraction(0)) / n
    ss = sum(((t - mu) * (t - mu) for t in v), Fraction(0))
    if n == 1:
        return Fraction(0)
    return ss / (n if norm_type == 1 else n - 1)


@pytest.mark.parametrize("dtype,npt", [("f32", np.float32), ("f64", np.float64)])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 200])
def test_var_brute_force(dtype, npt, n):
    g = np.random.default_rng(1000 + n)
    x = (g.standard_normal(n) * 3.0 + 7.0).astype(npt)
    for nt in (0, 1):
        assert rd.var(x, dtype, nt) == _brute_var(x, nt)


def test_var_closed_forms():
    # 1, 2, ..., n: variance n (n + 1) / 12 (normalised by n - 1), (n^2 - 1) / 12 by n
    for n in (2, 5, 100, 4097):
        x = np.arange(1, n + 1, dtype=np.float64)
        assert rd.var(x, "f64") == Fraction(n * (n + 1), 12)
        assert rd.var(x, "f64", 1) == Fraction(n * n - 1, 12)
    # constant: 0; one element: 0 under either normalisation
    assert rd.var(np.full(33, 2.5, np.float32), "f32") == 0
    assert rd.var(np.array([3.0], np.float32), "f32") == 0
    assert rd.var(np.array([3.0], np.float32), "f32", 1) == 0
    # two values a, b: (a - b)^2 / 2 by n - 1
    assert rd.var(np.array([1.0, 4.0]), "f64") == Fraction(9, 2)


def test_var_invariances():
    g = np.random.default_rng(5)
    x = g.integers(-1000, 1000, 513).astype(np.float64)
    v = rd.var(x, "f64")
    # shift by a large constant (exact in binary64): unchanged, with no cancellation
    assert rd.var(x + 2.0 ** 40, "f64") == v
    # scale by 2^k: times 4^k
    assert rd.var(x * 8.0, "f64") == v * 64
    # order does not matter
    assert rd.var(x[::-1].copy(), "f64") == v


def test_var_against_numpy():
    g = np.random.default_rng(9)
    x = g.lognormal(0.0, 1.0, 100_000).astype(np.float32)
    want = np.var(x.astype(np.float64), ddof=1)
    assert abs(float(rd.var(x, "f32")) - want) <= 1e-12 * want
    assert abs(float(rd.var(x, "f32", 1)) - np.var(x.astype(np.float64))) <= 1e-12 * want


def test_mean_dim_and_var_dim():
    g = np.random.default_rng(11)
    X = g.standard_normal((37, 23)).astype(np.float32)
    for dim in (0, 1):
        m = rd.mean_dim(X, dim, "f32")
        v = rd.var_dim(X, dim, "f32")
        v1 = rd.var_dim(X, dim, "f32", 1)
        groups = [X[:, j] for j in range(23)] if dim == 0 else [X[i, :] for i in range(37)]
        assert len(m) == len(groups) == len(v)
        for q, w, w1, grp in zip(m, v, v1, groups):
            assert q == rd.mean(grp, "f32")
            assert w == _brute_var(grp) and w1 == _brute_var(grp, 1)
        axis = 0 if dim == 0 else 1
        np.testing.assert_allclose([float(q) for q in m], X.astype(np.float64).mean(axis=axis), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose([float(q) for q in v], X.astype(np.float64).var(axis=axis, ddof=1), rtol=1e-12)
    # arithmetic columns: mean = (first + last) / 2
    A = np.arange(12, dtype=np.float64).reshape(4, 3, order="F")
    assert rd.mean_dim(A, 0, "f64") == [Fraction(3, 2), Fraction(11, 2), Fraction(19, 2)]
    assert rd.var_dim(A, 1, "f64") == [Fraction(16)] * 4          # rows k, k + 4, k + 8


def test_empty_and_degenerate_counts():
    E = np.zeros((0, 4), np.float32)
    assert rd.mean_dim(E, 0, "f32") == [None] * 4
    assert rd.var_dim(E, 0, "f32") == [None] * 4
    assert rd.mean_dim(E, 1, "f32") == []
    R = np.array([[1.0, 2.0, 4.0]], np.float32)                  # one row: var along dim 0 is 0
    assert rd.var_dim(R, 0, "f32") == [0, 0, 0]
    with pytest.raises(ValueError):
        rd.var(np.zeros(0, np.float32), "f32")
    with pytest.raises(ValueError):
        rd.var(np.array([1, 2], np.int32), "s32")
    # values whose squares leave binary32's range: (a - (-a))^2 / 2 = 2 a^2, exactly
    a = Fraction(float(np.float32(1e30)))
    assert rd.var(np.array([1e30, -1e30], np.float32), "f32") == 2 * a * a
