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
