"""The oracle's min / max / mean / 1-norm / infinity norm pinned by closed forms and
special cases."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import reduce as rd


def test_closed_forms():
    n = 1000
    x = np.arange(n, dtype=np.float32) - 300          # -300 .. 699
    assert rd.vmax(x, "f32") == 699.0 and rd.vmin(x, "f32") == -300.0
    assert rd.mean(x, "f32") == Fraction(699 - 300, 2)  # mean of an arithmetic progression
    assert rd.norm1(x, "f32") == sum(abs(v) for v in range(-300, 700))
    assert rd.norm_inf(x, "f32") == 699.0
    assert rd.norm_inf(-x, "f32") == 699.0
    y = np.array([1, 1, 2], np.float64)
    assert rd.mean(y, "f64") == Fraction(4, 3)
    assert rd.round_exact(rd.mean(y, "f64"), "f64") == 4 / 3


def test_integers():
    a = np.array([5, -7, 3], np.int32)
    assert rd.vmax(a, "s32") == 5 and rd.vmin(a, "s32") == -7
    u = np.array([0, 4294967295, 7], np.uint32)
    assert rd.vmax(u, "u32") == 4294967295 and rd.vmin(u, "u32") == 0
    with pytest.raises(ValueError):
        rd.mean(a, "s32")


def test_nan_and_empty():
    x = np.array([1.0, np.nan, -5.0], np.float32)
    assert math.isnan(rd.vmax(x, "f32")) and math.isnan(rd.vmin(x, "f32")) and math.isnan(rd.norm_inf(x, "f32"))
    assert rd.norm_inf(np.zeros((0, 3), np.float32), "f32") == 0.0
    with pytest.raises(ValueError):
        rd.vmax(np.zeros((0, 1), np.float32), "f32")
    inf = np.array([np.inf, -np.inf, 1.0], np.float64)
    assert rd.vmax(inf, "f64") == math.inf and rd.vmin(inf, "f64") == -math.inf


def test_exactness_where_float_sums_fail():
    # 2^24 + 1 + 1 ... : a float32 running sum would stall; the exact mean does not
    x = np.array([2.0 ** 24] + [1.0] * 8, np.float32)
    assert rd.mean(x, "f32") == Fraction(2 ** 24 + 8, 9)
    assert rd.norm1(-x, "f32") == 2 ** 24 + 8
