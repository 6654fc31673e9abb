"""min / max / mean / 1-norm / infinity norm, fused with the expression, against the
oracle: min, max and the infinity norm are element values (bit-exact); mean and the
1-norm come from the compensated sum (fp32 within 1e-6 relative, fp64 within
1e-12, 16-bit types within 1 ulp of the exact value rounded to the type)."""
import math

import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from oracle import reduce as rd

pytestmark = pytest.mark.gpu

Z_POST = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",), ("load", 3),
          ("trans",), ("sub",)]
W_POST = [("load", 0), ("exp",), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]
REL = {"f32": 1e-6, "f64": 1e-12}


@pytest.fixture(scope="module")
def coot():
    import torch
    import paper_2508_11385_amd as coot
    coot.init(0)
    torch.cuda.synchronize()
    return coot


def up(coot, a, dtype):
    return coot.Mat.from_numpy(a, dtype=dtype)


def _scalar(m):
    return float(m.numpy().ravel()[0])


def _same(got, want):
    return (math.isnan(got) and math.isnan(want)) or got == want


def _close(got, exact, dtype, scale):
    if dtype in REL:
        assert rd.rel_err(got, exact, scale) <= REL[dtype], (got, float(exact))
    else:
        want = rd.round_exact(exact, dtype)
        w = np.array([want], np.float64)
        g = np.array([got], np.float64)
        if dtype == "f16":
            d = abs(int(g.astype(np.float16).view(np.int16)[0]) - int(w.astype(np.float16).view(np.int16)[0]))
        else:
            d = abs(int(g.astype(np.float32).view(np.int32)[0] >> 16) - int(w.astype(np.float32).view(np.int32)[0] >> 16))
        assert d <= 1, (got, want)


@pytest.mark.parametrize("dtype", ["f32", "f64", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1), (67, 45), (1000, 3), (130, 257)])
def test_float_reductions(coot, dtype, shape):
    r, c = shape
    A, B, C, D = synth.matrix_inputs(n_rows=r, n_cols=c, dtype=dtype)
    gA, gB, gC, gD = (up(coot, x, dtype) for x in (A, B, C, D))
    Zo = ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype)
    Wo = ew.evaluate(W_POST, [A, B], [1.0], dtype)
    for e, ref in ((2.0 * gA + gB % gC - coot.trans(gD), Zo), (coot.exp(gA) / (1.0 + coot.abs(gB)), Wo)):
        assert _same(_scalar(coot.max(e)), rd.vmax(ref, dtype))
        assert _same(_scalar(coot.min(e)), rd.vmin(ref, dtype))
        assert _same(_scalar(coot.norm_inf(e)), rd.norm_inf(ref, dtype))
        scale = rd.sum_abs(ref)
        _close(_scalar(coot.mean(e)), rd.mean(ref, dtype), dtype, scale / ref.size)
        _close(_scalar(coot.norm1(e)), rd.norm1(ref, dtype), dtype, scale)


@pytest.mark.parametrize("dtype", ["u32", "s32"])
def test_integer_extremes(coot, dtype):
    import paper_2508_11385_amd._coot as cc
    g = synth.rng_for(81)
    lo, hi = (0, 1 << 32) if dtype == "u32" else (-(1 << 31), 1 << 31)
    A = synth.uniform_int(g, (300, 77), dtype, lo, hi)
    B = synth.uniform_int(g, (77, 300), dtype, lo, hi)
    gA, gB = up(coot, A, dtype), up(coot, B, dtype)
    post = [("load", 0), ("load", 1), ("trans",), ("sub",)]
    ref = ew.evaluate(post, [A, B], [], dtype)
    e = gA - coot.trans(gB)
    assert int(coot.max(e).numpy().ravel()[0]) == rd.vmax(ref, dtype)
    assert int(coot.min(e).numpy().ravel()[0]) == rd.vmin(ref, dtype)
    assert int(coot.max(gA).numpy().ravel()[0]) == rd.vmax(A, dtype)
    for f in (coot.mean, coot.norm1, coot.norm_inf):
        with pytest.raises(cc.CootError) as err:
            f(gA)
        assert err.value.status == cc.COOT_ETYPE


def test_nan_empty_and_infinities(coot):
    import paper_2508_11385_amd._coot as cc
    A = synth.uniform(synth.rng_for(82), (100, 40), "f32")
    A[37, 5] = np.nan
    gA = up(coot, A, "f32")
    for f in (coot.max, coot.min, coot.norm_inf, coot.mean, coot.norm1):
        assert math.isnan(_scalar(f(gA))), f.__name__
    B = synth.uniform(synth.rng_for(83), (100, 40), "f32")
    B[3, 3], B[4, 4] = np.inf, -np.inf
    gB = up(coot, B, "f32")
    assert _scalar(coot.max(gB)) == math.inf and _scalar(coot.min(gB)) == -math.inf
    assert _scalar(coot.norm_inf(gB)) == math.inf
    E = up(coot, np.zeros((0, 5), np.float32), "f32")
    for f in (coot.max, coot.min, coot.mean):
        with pytest.raises(cc.CootError) as err:
            f(E)
        assert err.value.status == cc.COOT_EINVAL
    assert _scalar(coot.norm_inf(E)) == 0.0 and _scalar(coot.norm1(E)) == 0.0


def test_fused_equals_unfused_and_full_size(coot):
    A, B, C, D = synth.matrix_inputs(4096, "f32")
    gA, gB, gC, gD = (up(coot, x, "f32") for x in (A, B, C, D))
    e = 2.0 * gA + gB % gC - coot.trans(gD)
    for f in (coot.max, coot.min, coot.norm_inf):
        assert _scalar(f(e)) == _scalar(f(e, unfused=True))
    Zo = ew.evaluate(Z_POST, [A, B, C, D], [2.0], "f32")
    assert _scalar(coot.max(e)) == rd.vmax(Zo, "f32") and _scalar(coot.min(e)) == rd.vmin(Zo, "f32")
    scale = rd.sum_abs(Zo)
    assert rd.rel_err(_scalar(coot.mean(e)), rd.mean(Zo, "f32"), scale / Zo.size) <= 1e-6
    assert rd.rel_err(_scalar(coot.norm1(e)), rd.norm1(Zo, "f32"), scale) <= 1e-6
