"""Edge values through the fp32 / fp64 kernels, against the oracle (IEEE semantics:
round-to-nearest-even, subnormals kept, signed zeros, infinities, NaN propagation).

Every operator is correctly rounded on the device except log (binary32: the
library's own table method, within 1 ulp; binary64: the device math library's,
faithful): results must have the oracle's bits (any NaN matches any NaN), log
within 1 ulp.  Covers every pair of edge values through each binary operator, each
unary operator, exp at its overflow and underflow thresholds, the 2-D workload
expressions Z = 2*A + B%C - trans(D) and W = exp(A) / (1 + abs(B)) over edge
operands, and log over wide magnitudes."""
import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from tests.exact import ulp_distance

pytestmark = pytest.mark.gpu

NPT = {"f32": np.float32, "f64": np.float64}
UT = {"f32": np.uint32, "f64": np.uint64}


@pytest.fixture(scope="module")
def coot():
    import torch
    import paper_2508_11385_amd as coot
    coot.init(0)
    torch.cuda.synchronize()
    return coot


def edge_values(dtype):
    t = NPT[dtype]
    fi = np.finfo(t)
    tiny_sub = fi.smallest_subnormal
    max_sub = t(fi.tiny) - tiny_sub
    base = [0.0, tiny_sub, max_sub, fi.tiny, 1.0, fi.max, np.inf, 0.5, 2.0, 3.0, np.nan]
    v = [t(x) for x in base] + [t(-x) for x in base[:-1]]
    # a quiet NaN with a payload and a negative quiet NaN
    nb = np.array([0x7FC01234 if dtype == "f32" else 0x7FF8000000001234,
                   0xFFC00000 if dtype == "f32" else 0xFFF8000000000000], dtype=UT[dtype])
    return np.concatenate([np.array(v, dtype=t), nb.view(t)])


def assert_bits(got, want, dtype, what, ulps=0):
    got = np.ascontiguousarray(got, NPT[dtype])
    want = np.ascontiguousarray(want, NPT[dtype])
    assert got.shape == want.shape, what
    nan = np.isnan(got) & np.isnan(want)
    same = got.view(UT[dtype]) == want.view(UT[dtype])
    if ulps:
        d = ulp_distance(got, want)
        zsign = (got == 0) & (want == 0) & (np.signbit(got) != np.signbit(want))
        ok = nan | same | ((d <= ulps) & ~zsign & ~np.isnan(got) & ~np.isnan(want))
    else:
        ok = nan | same
    if not ok.all():
        i = np.flatnonzero(~ok.ravel())[:5]
        raise AssertionError(f"{what}: {int((~ok).sum())} elements differ, e.g. got {got.ravel()[i]} "
                             f"want {want.ravel()[i]}")


def up(coot, a, kind=None):
    return coot.Mat.from_numpy(a, kind=kind)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_every_pair_of_edge_values(coot, dtype):
    v = edge_values(dtype)
    n = len(v)
    A = np.repeat(v[:, None], n, axis=1)          # A[i, j] = v[i]
    B = np.repeat(v[None, :], n, axis=0)          # B[i, j] = v[j]
    gA, gB = up(coot, A), up(coot, B)
    cases = [
        ([("load", 0), ("load", 1), ("add",)], gA + gB, [], 0),
        ([("load", 0), ("load", 1), ("sub",)], gA - gB, [], 0),
        ([("load", 0), ("load", 1), ("schur",)], gA % gB, [], 0),
        ([("load", 0), ("load", 1), ("div",)], gA / gB, [], 0),
        ([("load", 0), ("neg",)], -gA, [], 0),
        ([("load", 0), ("abs",)], coot.abs(gA), [], 0),
        ([("load", 0), ("neg",), ("abs",)], coot.abs(-gA), [], 0),
        ([("load", 0), ("sqrt",)], coot.sqrt(gA), [], 0),
        ([("load", 0), ("square",)], coot.square(gA), [], 0),
        ([("load", 0), ("exp",)], coot.exp(gA), [], 0),
        ([("load", 0), ("log",)], coot.log(gA), [], 1),
        ([("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("add",)], 0.001 * gA + gB, [0.001], 0),
        ([("load", 0), ("scalar", 0), ("sub",)], gA - 0.0, [0.0], 0),
        ([("scalar", 0), ("load", 0), ("sub",)], 0.0 - gA, [0.0], 0),
        ([("load", 0), ("load", 1), ("trans",), ("sub",)], gA - coot.trans(gB), [], 0),
    ]
    for post, e, sc, ulps in cases:
        got = coot.eval(e).numpy()
        ops = [A, B][:1 + any(p == ("load", 1) for p in post)]
        assert_bits(got, ew.evaluate(post, ops, sc, dtype), dtype, str(post), ulps)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_workload_expressions_over_edge_operands(coot, dtype):
    """Z and W with every operand drawn from the edge values (tiled and flat kernels)."""
    v = edge_values(dtype)
    g = synth.rng_for(81, 0 if dtype == "f32" else 1)
    r, c = 67, 45
    A, B, C = (v[g.integers(0, len(v), (r, c))] for _ in range(3))
    D = v[g.integers(0, len(v), (c, r))]
    gA, gB, gC, gD = (up(coot, x) for x in (A, B, C, D))
    Z = coot.eval(2.0 * gA + gB % gC - coot.trans(gD)).numpy()
    zp = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",), ("load", 3),
          ("trans",), ("sub",)]
    assert_bits(Z, ew.evaluate(zp, [A, B, C, D], [2.0], dtype), dtype, "Z")
    W = coot.eval(coot.exp(gA) / (1.0 + coot.abs(gB))).numpy()
    wp = [("load", 0), ("exp",), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]
    assert_bits(W, ew.evaluate(wp, [A, B], [1.0], dtype), dtype, "W")


EXP_EDGES = {
    # largest finite result, first overflow, smallest normal result, subnormal results, underflow to 0
    "f32": [88.72283, 88.722835, 88.72284, 89.0, -87.33654, -87.33655, -100.0, -103.27893, -103.972076, -103.97208,
            -103.972084, -104.0, 1e-8, -1e-8, 1e-30, 0.0, -0.0],
    "f64": [709.782712893384, 709.7827128933841, 710.0, -708.3964185322641, -708.39641853226, -740.0,
            -745.1332191019411, -745.1332191019412, -746.0, 1e-17, -1e-17, 1e-300, 0.0, -0.0],
}


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_exp_at_its_thresholds(coot, dtype):
    t = NPT[dtype]
    base = np.array(EXP_EDGES[dtype], dtype=t)
    # each threshold with its neighbours 1, 2 and 3 ulps away on both sides
    xs = [base]
    for k in (1, 2, 3):
        up_, dn = base.copy(), base.copy()
        for _ in range(k):
            up_ = np.nextafter(up_, t(np.inf))
            dn = np.nextafter(dn, t(-np.inf))
        xs += [up_, dn]
    x = np.concatenate(xs).reshape(-1, 1)
    got = coot.eval(coot.exp(up(coot, x, "col"))).numpy()
    assert_bits(got, ew.evaluate([("load", 0), ("exp",)], [x], [], dtype), dtype, "exp thresholds")
    # and through the tiled kernel (a transposed leaf)
    xt = np.ascontiguousarray(np.tile(x.T, (3, 1)))                    # 3 x n, read as trans -> n x 3
    got_t = coot.eval(coot.exp(coot.trans(up(coot, xt)))).numpy()
    assert_bits(got_t, ew.evaluate([("load", 0), ("trans",), ("exp",)], [xt], [], dtype), dtype, "exp tiled")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_log_within_one_ulp(coot, dtype):
    """log (COOT_OP_LOG) over magnitudes from the smallest subnormal to the largest
    finite value, random bit patterns, values next to 1, and in a tree."""
    t = NPT[dtype]
    g = synth.rng_for(82, 0 if dtype == "f32" else 1)
    lim = 87 if dtype == "f32" else 700
    ut = UT[dtype]
    bits = g.integers(0, np.iinfo(np.int32 if dtype == "f32" else np.int64).max, 1 << 16, dtype=np.int64)
    rnd = bits.astype(ut).view(t)
    near1 = (1.0 + (np.arange(-200, 200) * float(np.finfo(t).eps))).astype(t)
    x = np.concatenate([np.exp(g.uniform(-lim, lim, 1 << 16)).astype(t), rnd, near1,
                        np.array([np.finfo(t).smallest_subnormal, np.finfo(t).tiny, np.finfo(t).max, 1.0, 2.0, 0.5,
                                  10.0], dtype=t)])
    x = x[np.isfinite(x) & (x > 0)].reshape(-1, 1)
    got = coot.eval(coot.log(up(coot, x, "col"))).numpy()
    assert_bits(got, ew.evaluate([("load", 0), ("log",)], [x], [], dtype), dtype, "log", ulps=1)
    # log inside an expression: log(1 + abs(A)) - B over the 2-D workload's shape class
    A, B = synth.uniform(g, (130, 257), dtype, -50, 50), synth.uniform(g, (130, 257), dtype)
    got = coot.eval(coot.log(1.0 + coot.abs(up(coot, A))) - up(coot, B)).numpy()
    post = [("scalar", 0), ("load", 0), ("abs",), ("add",), ("log",), ("load", 1), ("sub",)]
    want = ew.evaluate(post, [A, B], [1.0], dtype)
    # one faithful log feeds one exact subtraction: 1 ulp of the log can become more
    # ulps of a difference near 0, so compare the log's own output here
    got_log = coot.eval(coot.log(1.0 + coot.abs(up(coot, A)))).numpy()
    assert_bits(got_log, ew.evaluate(post[:5], [A], [1.0], dtype), dtype, "log(1 + |A|)", ulps=1)
    d = ulp_distance(got, want)
    assert np.isfinite(got).all() and np.median(d) == 0
