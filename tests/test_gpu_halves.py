"""16-bit storage types (f16, bf16) on the HIP path against the oracle.

Every operator computes in binary32 and is rounded to the storage type, which
for f16 is the correctly rounded result of every operator here (exp included,
binary32's exp being correctly rounded) and for bf16 too while the binary32
result is normal: 0 ulp expected, 1 ulp allowed for bf16 results below 2^-126.
Reductions accumulate in compensated binary32 and round once to the type:
within 1 ulp of the exact sum rounded to the type."""
import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from oracle import reduce as rd

pytestmark = pytest.mark.gpu

Z_POST = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",), ("load", 3),
          ("trans",), ("sub",)]
W_POST = [("load", 0), ("exp",), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]
HALVES = ["f16", "bf16"]


@pytest.fixture(scope="module")
def coot():
    import torch
    import paper_2508_11385_amd as coot
    coot.init(0)
    torch.cuda.synchronize()
    return coot


def up(coot, a, dtype, kind=None):
    return coot.Mat.from_numpy(a, dtype=dtype, kind=kind)


def _ordered(a, dtype):
    """16-bit patterns as integers ordered like the values (sign-magnitude -> two's complement)."""
    a = np.asarray(a)
    if dtype == "f16":
        b = a.astype(np.float16).view(np.uint16).astype(np.int64)
    else:
        b = (a.astype(np.float32).view(np.uint32) >> 16).astype(np.int64)
    return np.where(b & 0x8000, -(b & 0x7FFF), b)


def ulp16(got, want, dtype):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    d = np.abs(_ordered(got, dtype) - _ordered(want, dtype))
    d[np.isnan(got) & np.isnan(want)] = 0
    return d


def assert_exact(got, want, dtype, what):
    d = ulp16(got, want, dtype)
    allowed = np.zeros(d.shape, np.int64)
    if dtype == "bf16":
        allowed[np.abs(np.asarray(want, np.float64)) < 2.0 ** -126] = 1
    bad = d > allowed
    assert not bad.any(), f"{what}: {int(bad.sum())} elements off, worst {int(d.max())} ulp"


def _z(coot, A, B, C, D):
    return 2.0 * A + B % C - coot.trans(D)


def _w(coot, A, B):
    return coot.exp(A) / (1.0 + coot.abs(B))


@pytest.mark.parametrize("dtype", HALVES)
@pytest.mark.parametrize("shape", [(1, 1), (3, 5), (64, 64), (67, 45), (130, 257), (1000, 3)])
def test_Z_and_W_elementwise(coot, dtype, shape):
    r, c = shape
    A, B, C, D = synth.matrix_inputs(n_rows=r, n_cols=c, dtype=dtype)
    gA, gB, gC, gD = (up(coot, x, dtype) for x in (A, B, C, D))
    Z = coot.eval(_z(coot, gA, gB, gC, gD)).numpy()
    W = coot.eval(_w(coot, gA, gB)).numpy()
    assert_exact(Z, ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype), dtype, "Z")
    assert_exact(W, ew.evaluate(W_POST, [A, B], [1.0], dtype), dtype, "W")


@pytest.mark.parametrize("dtype", HALVES)
def test_random_trees(coot, dtype):
    g = synth.rng_for(71, 0 if dtype == "f16" else 1)
    for _ in range(60):
        r, c = int(g.integers(1, 70)), int(g.integers(1, 70))
        spec = synth.random_tree(g, int(g.integers(1, 7)), int(g.integers(1, 5)), r, c, dtype)
        ops = synth.operands_for(spec, g)
        mats = [up(coot, o, dtype) for o in ops]
        st = []
        for it in spec.postfix:
            if it[0] == "load":
                st.append(mats[it[1]])
            elif it[0] == "scalar":
                st.append(coot.Scalar(spec.scalars[it[1]]))
            elif it[0] in ("add", "sub", "schur", "div"):
                b, a = st.pop(), st.pop()
                st.append(coot.Node(it[0], [a, b]))
            else:
                st.append(coot.Node(it[0], [st.pop()]))
        got = coot.eval(st[0]).numpy()
        assert_exact(got, ew.evaluate(spec.postfix, ops, spec.scalars, dtype), dtype, str(spec.postfix))


@pytest.mark.parametrize("dtype", HALVES)
@pytest.mark.parametrize("shape", [(67, 45), (130, 257), (1000, 3)])
def test_reductions(coot, dtype, shape):
    r, c = shape
    A, B, C, D = synth.matrix_inputs(n_rows=r, n_cols=c, dtype=dtype)
    gA, gB, gC, gD = (up(coot, x, dtype) for x in (A, B, C, D))
    Zo = ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype)
    gZ = up(coot, Zo, dtype)

    def close(got, exact, what):
        want = np.array([rd.round_exact(q, dtype) for q in exact])
        d = ulp16(np.asarray(got).ravel(), want, dtype)
        assert d.max() <= 1, f"{what}: worst {int(d.max())} ulp"

    close(coot.accu(_z(coot, gA, gB, gC, gD)).numpy(), [rd.accu(Zo, dtype)], "accu fused")
    close(coot.accu(gZ).numpy(), [rd.accu(Zo, dtype)], "accu")
    for dim in (0, 1):
        ex = rd.sum_dim(Zo, dim, dtype)
        close(coot.sum(_z(coot, gA, gB, gC, gD), dim).numpy(), ex, f"fused sum dim {dim}")
        close(coot.sum(gZ, dim).numpy(), ex, f"sum dim {dim}")
    close(coot.dot(gA, gB).numpy(), [rd.dot(A, B, dtype)], "dot")
    nrm = rd.norm(A, dtype)
    got = float(coot.norm(gA).numpy()[0, 0])
    assert ulp16([got], ew.round_to(np.array([nrm]), dtype), dtype).max() <= 1, "norm"


@pytest.mark.parametrize("dtype", HALVES)
def test_fused_equals_unfused(coot, dtype):
    A, B, C, D = synth.matrix_inputs(n_rows=130, n_cols=257, dtype=dtype)
    gA, gB, gC, gD = (up(coot, x, dtype) for x in (A, B, C, D))
    for e in (_z(coot, gA, gB, gC, gD), _w(coot, gA, gB)):
        fused = coot.eval(e).numpy()
        unfused = coot.eval(e, unfused=True).numpy()
        assert np.array_equal(fused.view(np.uint16) if dtype == "f16" else fused.view(np.uint32),
                              unfused.view(np.uint16) if dtype == "f16" else unfused.view(np.uint32))


@pytest.mark.parametrize("dtype", HALVES)
def test_full_size_sampled(coot, dtype):
    A, B, C, D = synth.matrix_inputs(4096, dtype)
    gA, gB, gC, gD = (up(coot, x, dtype) for x in (A, B, C, D))
    Z = coot.eval(_z(coot, gA, gB, gC, gD)).numpy()
    W = coot.eval(_w(coot, gA, gB)).numpy()
    g = np.random.default_rng(17)
    rows, cols = g.integers(0, 4096, 50_000), g.integers(0, 4096, 50_000)
    assert_exact(Z[rows, cols], ew.evaluate_at(Z_POST, [A, B, C, D], [2.0], dtype, rows, cols), dtype, "Z")
    assert_exact(W[rows, cols], ew.evaluate_at(W_POST, [A, B], [1.0], dtype, rows, cols), dtype, "W")


def test_halves_outside_batches_and_cost_model(coot):
    import paper_2508_11385_amd._coot as cc
    A = up(coot, np.ones((4, 4), np.float16), "f16")
    with pytest.raises(cc.CootError) as e:
        coot.Batch([(A + A, None)])
    assert e.value.status == cc.COOT_EUNSUPPORTED
    h = coot.frontend.compiled(coot.flatten(A + A))
    with pytest.raises(cc.CootError) as e:
        cc.coot_costmodel_features(h, 4, 4, 0, [(4, 1, 4, 4)])
    assert e.value.status == cc.COOT_EUNSUPPORTED


def _edge_values(dtype):
    """Finite extremes, subnormals, zeros of both signs, infinities and NaN of the type."""
    if dtype == "f16":
        bits = [0x0000, 0x8000, 0x3C00, 0xBC00, 0x7BFF, 0xFBFF, 0x0400, 0x0001, 0x0003, 0x03FF, 0x2E66, 0x63D0,
                0x7C00, 0xFC00, 0x7E00]
        return np.array(bits, np.uint16).view(np.float16)
    bits = [0x0000, 0x8000, 0x3F80, 0xBF80, 0x7F7F, 0xFF7F, 0x0080, 0x0001, 0x0003, 0x007F, 0x3DCD, 0x7149,
            0x7F80, 0xFF80, 0x7FC0]
    return (np.array(bits, np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("dtype", HALVES)
def test_special_values(coot, dtype):
    """Every pair of edge values through each operator: overflow to infinity, gradual
    underflow, signed zeros, NaN propagation, as the oracle rounds them."""
    v = _edge_values(dtype)
    n = len(v)
    A = np.repeat(v[:, None], n, axis=1)
    B = np.repeat(v[None, :], n, axis=0)
    gA, gB = up(coot, A, dtype), up(coot, B, dtype)
    cases = [
        ([("load", 0), ("load", 1), ("add",)], gA + gB, []),
        ([("load", 0), ("load", 1), ("sub",)], gA - gB, []),
        ([("load", 0), ("load", 1), ("schur",)], gA % gB, []),
        ([("load", 0), ("load", 1), ("div",)], gA / gB, []),
        ([("load", 0), ("sqrt",)], coot.sqrt(gA), []),
        ([("load", 0), ("exp",)], coot.exp(gA), []),
        ([("load", 0), ("log",)], coot.log(gA), []),
        ([("load", 0), ("square",)], coot.square(gA), []),
        ([("load", 0), ("neg",), ("abs",)], coot.abs(-gA), []),
        ([("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("add",)], 0.001 * gA + gB, [0.001]),
        ([("load", 0), ("scalar", 0), ("schur",)], gA * 1e-3, [1e-3]),
    ]
    for post, e, sc in cases:
        got = coot.eval(e).numpy()
        want = ew.evaluate(post, [A, B][:1 + any(p == ("load", 1) for p in post)], sc, dtype)
        assert_exact(got, want, dtype, str(post))


@pytest.mark.parametrize("dtype", HALVES)
@pytest.mark.parametrize("cfg", [(8, 1, 4, 4), (8, 4, 2, 8), (8, 1, 4, 16), (4, 2, 8, 2)])
def test_sixteen_byte_groups(coot, dtype, cfg):
    """vec 8: 16-byte accesses of 16-bit elements, flat and tiled, ragged shapes."""
    for r, c in ((130, 257), (1000, 3), (64, 64)):
        A, B, C, D = synth.matrix_inputs(n_rows=r, n_cols=c, dtype=dtype)
        gA, gB, gC, gD = (up(coot, x, dtype) for x in (A, B, C, D))
        Z = coot.eval(_z(coot, gA, gB, gC, gD), cfg=cfg).numpy()
        W = coot.eval(_w(coot, gA, gB), cfg=cfg).numpy()
        assert_exact(Z, ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype), dtype, f"Z {cfg}")
        assert_exact(W, ew.evaluate(W_POST, [A, B], [1.0], dtype), dtype, f"W {cfg}")
        s0 = coot.sum(_z(coot, gA, gB, gC, gD), 0, cfg=cfg).numpy().ravel()
        want = [rd.round_exact(q, dtype) for q in rd.sum_dim(ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype), 0, dtype)]
        assert ulp16(s0, want, dtype).max() <= 1


@pytest.mark.parametrize("dtype", HALVES)
@pytest.mark.parametrize("shape", [(128, 96), (67, 45), (130, 257)])
def test_dim_reductions_four_transposed_leaves(coot, dtype, shape):
    """Four transposed 16-bit leaves stage through 32 x 32 tiles; the dimension sums,
    means and variances (16-byte groups requested: planned as 4-element groups, the
    widest a 32 x 32 tile of 256 threads covers) against the oracle on aligned and
    ragged shapes."""
    r, c = shape
    g = synth.rng_for(71, r, c)
    A = synth.uniform(g, (r, c), dtype)
    Ts = [synth.uniform(g, (c, r), dtype) for _ in range(4)]
    post = [("load", 0)]
    for k in range(4):
        post += [("load", k + 1), ("trans",), ("add",)]
    ref = ew.evaluate(post, [A] + Ts, [], dtype)
    gA = up(coot, A, dtype)
    gT = [up(coot, t, dtype) for t in Ts]

    def e():
        x = gA
        for t in gT:
            x = x + coot.trans(t)
        return x

    def close(got, exact, what):
        want = np.array([rd.round_exact(q, dtype) for q in exact])
        d = ulp16(np.asarray(got).ravel(), want, dtype)
        assert d.max() <= 1, f"{what}: worst {int(d.max())} ulp"

    for cfg in (None, (8, 0, 0, 0)):
        for dim in (0, 1):
            close(coot.sum(e(), dim, cfg=cfg).numpy(), rd.sum_dim(ref, dim, dtype), f"sum dim {dim} {cfg}")
            close(coot.mean(e(), dim=dim, cfg=cfg).numpy(), rd.mean_dim(ref, dim, dtype), f"mean dim {dim} {cfg}")
            v = coot.var(e(), dim=dim, cfg=cfg).numpy().ravel()
            close(v, rd.var_dim(ref, dim, dtype, 0), f"var dim {dim} {cfg}")
