"""The kernels' exponential (csrc/device/coot_exp.h) compiled for the host with
g++ and compared with the oracle's correctly rounded exp on a large sample
(binary32 and binary64, edges included).  The GPU parity tests check the device
build of the same code; this test pins its arithmetic without a GPU."""
import numpy as np
import pytest

from oracle import elementwise as ew
from tests import hostexp


@pytest.fixture(scope="module")
def lib():
    L = hostexp.build()
    if L is None:
        pytest.skip("g++ not available")
    return L


def test_binary32_sample(lib):
    rng = np.random.default_rng(31)
    bits = rng.integers(0, 1 << 32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    x = np.concatenate([bits.view(np.float32), rng.uniform(-104, 89, 1 << 18).astype(np.float32),
                        np.array([0, -0.0, 88.72283, 88.72284, 88.7228394, -87.33655, -103.27893, -103.97208,
                                  -103.972084, -104, 1e-8, -1e-8, np.inf, -np.inf, np.nan], np.float32)])
    y = np.empty_like(x)
    lib.expf_n(x.ctypes.data, y.ctypes.data, x.size)
    want = ew.exp_rounded(x, "f32")
    both_nan = np.isnan(y) & np.isnan(want)
    assert np.all((y.view(np.uint32) == want.view(np.uint32)) | both_nan)


def test_binary64_sample(lib):
    rng = np.random.default_rng(32)
    x = np.concatenate([rng.uniform(-1, 1, 1 << 17), rng.uniform(-746, 710, 1 << 17), rng.uniform(-1e-3, 1e-3, 1 << 14),
                        np.array([0.0, 709.782712893384, 709.7827128933841, -745.1332191019411, -745.1332191019412,
                                  -708.396418532264, np.inf, -np.inf])])
    y = np.empty_like(x)
    lib.exp_n(x.ctypes.data, y.ctypes.data, x.size)
    want = ew.exp_rounded(x, "f64")
    assert np.array_equal(y, want)


def test_binary32_two_level_path(lib):
    """exp_rn<float>: the fast path (double-word arithmetic in binary32 words) with its
    ambiguity test, plus the exact slow path for the lanes it rejects, on a sample
    dense in the fast range."""
    rng = np.random.default_rng(33)
    bits = rng.integers(0, 1 << 32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    x = np.concatenate([bits.view(np.float32), rng.uniform(-86, 88, 1 << 20).astype(np.float32),
                        rng.uniform(-1e-3, 1e-3, 1 << 16).astype(np.float32),
                        np.array([0, -0.0, -86, 88, -85.99999, 87.99999, 88.72283, -87.33655, -103.97208,
                                  np.inf, -np.inf, np.nan], np.float32)])
    y = np.empty_like(x)
    lib.expf_rn_n(x.ctypes.data, y.ctypes.data, x.size)
    want = ew.exp_rounded(x, "f32")
    both_nan = np.isnan(y) & np.isnan(want)
    assert np.all((y.view(np.uint32) == want.view(np.uint32)) | both_nan)
    # the fast path decides nearly every lane of its range (rejections about 1 in 10^4)
    inr = rng.uniform(-86, 88, 1 << 20).astype(np.float32)
    assert lib.expf_fast_misses(inr.ctypes.data, inr.size) <= 1000


def test_binary64_two_level_path(lib):
    rng = np.random.default_rng(34)
    x = np.concatenate([rng.uniform(-1, 1, 1 << 17), rng.uniform(-708, 709, 1 << 17),
                        np.array([0.0, -707.0, 709.0, 709.782712893384, -745.1332191019411, np.inf, -np.inf])])
    y = np.empty_like(x)
    lib.exp_rn_n(x.ctypes.data, y.ctypes.data, x.size)
    want = ew.exp_rounded(x, "f64")
    assert np.array_equal(y, want)


def _ulps32(a, b):
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


def test_binary32_log_sample(lib):
    """log_lf (the kernels' binary32 log, float-float arithmetic only) against the
    oracle's correctly rounded log: at most 1 ulp, almost always 0; specials exact."""
    rng = np.random.default_rng(34)
    bits = rng.integers(0, 1 << 32, size=1 << 20, dtype=np.uint64).astype(np.uint32)
    near1 = (1.0 + np.arange(-3000, 3000) * float(np.finfo(np.float32).eps)).astype(np.float32)
    x = np.concatenate([bits.view(np.float32), np.exp(rng.uniform(-103, 88.7, 1 << 18)).astype(np.float32), near1,
                        np.array([0.0, -0.0, 1.0, 2.0, 0.5, np.inf, -np.inf, np.nan, -1.0, 1e-45, 1.1754942e-38,
                                  1.17549435e-38, 3.4028235e38, 0.70710677, 0.70710683, 1.4142135, 1.4142137],
                                 np.float32)])
    y = np.empty_like(x)
    lib.logf_n(x.ctypes.data, y.ctypes.data, x.size)
    with np.errstate(all="ignore"):
        want = ew.log_rounded(x, "f32")
    special = ~np.isfinite(want)
    assert np.all((y[special] == want[special]) | (np.isnan(y[special]) & np.isnan(want[special])))
    d = _ulps32(y[~special], want[~special])
    assert d.max() <= 1
    assert (d > 0).sum() <= 4, f"{(d > 0).sum()} of {d.size} not correctly rounded"
