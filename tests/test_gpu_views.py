"""Index maps beyond transpose: broadcast columns / rows (each_col, each_row: a column
stride of 0) and the diagonal view (elements ld + 1 apart), read and written through
the fused kernels, against the oracle on the materialised operands."""
import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from oracle import reduce as rd
from tests.exact import ulp_distance

REL = {"f32": 1e-6, "f64": 1e-12}

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def coot():
    import torch
    import paper_2508_11385_amd as coot
    coot.init(0)
    torch.cuda.synchronize()
    return coot


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(70, 50), (1, 9), (129, 3), (256, 256)])
def test_each_col_and_each_row(coot, dtype, shape):
    r, c = shape
    g = synth.rng_for(91, r, c)
    X = synth.uniform(g, (r, c), dtype)
    v = synth.uniform(g, (r, 1), dtype)
    w = synth.uniform(g, (1, c), dtype)
    gX = coot.Mat.from_numpy(X)
    gv = coot.Mat.from_numpy(v, kind="col")
    gw = coot.Mat.from_numpy(w, kind="row")
    V = np.repeat(v, c, axis=1)              # the broadcasts, materialised for the oracle
    Wm = np.repeat(w, r, axis=0)
    got = coot.eval(2.0 * (gX.each_col() + gv) - gX.each_row() % gw).numpy()
    post = [("scalar", 0), ("load", 0), ("load", 1), ("add",), ("schur",), ("load", 0), ("load", 2), ("schur",),
            ("sub",)]
    want = ew.evaluate(post, [X, V, Wm], [2.0], dtype)
    assert np.max(ulp_distance(got, want)) == 0
    # fused with its reductions
    s0 = coot.sum(gX.each_col() / (1.0 + coot.abs(gv)), 0).numpy().ravel()
    post2 = [("load", 0), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]
    ref = ew.evaluate(post2, [X, V], [1.0], dtype)
    tol = 1e-6 if dtype == "f32" else 1e-12
    for j in range(c):
        assert rd.rel_err(float(s0[j]), rd.exact_sum(ref[:, j]), rd.sum_abs(ref[:, j])) <= tol
    assert float(coot.max(gX.each_row() - gw).numpy()[0, 0]) == rd.vmax(ew.evaluate(
        [("load", 0), ("load", 1), ("sub",)], [X, Wm], [], dtype), dtype)


def test_each_col_in_place_and_diag(coot):
    g = synth.rng_for(92)
    X = synth.uniform(g, (40, 40), "f32")
    v = synth.uniform(g, (40, 1), "f32")
    gX = coot.Mat.from_numpy(X)
    gv = coot.Mat.from_numpy(v, kind="col")
    each = gX.each_col()
    each -= gv
    want = ew.evaluate([("load", 0), ("load", 1), ("sub",)], [X, np.repeat(v, 40, axis=1)], [], "f32")
    assert np.array_equal(gX.numpy(), want)
    # the diagonal: read (trace), then updated in place
    tr = float(coot.accu(gX.diag()).numpy()[0, 0])
    assert rd.rel_err(tr, rd.exact_sum(np.diag(want)), rd.sum_abs(np.diag(want))) <= 1e-6
    d = gX.diag()
    d += 100.0
    expect = want.copy()
    idx = np.arange(40)
    expect[idx, idx] = ew.evaluate([("load", 0), ("scalar", 0), ("add",)], [np.diag(want).reshape(1, -1)],
                                   [100.0], "f32").ravel()
    assert np.array_equal(gX.numpy(), expect)
    # a rectangular matrix's diagonal has min(n_rows, n_cols) elements
    R = coot.Mat.from_numpy(synth.uniform(g, (7, 3), "f32"))
    assert R.diag().n_cols == 3 and np.array_equal(coot.eval(R.diag()).numpy().ravel(), np.diag(R.numpy()))


def test_broadcast_errors(coot):
    import paper_2508_11385_amd._coot as cc
    gv = coot.Mat.from_numpy(np.ones((8, 1), np.float32), kind="col")
    b = coot.bcast_col(gv, 5)
    X = coot.Mat.from_numpy(np.ones((8, 5), np.float32))
    with pytest.raises(cc.CootError) as e:           # a broadcast operand is never written
        coot.eval(X + 1.0, out=b)
    assert e.value.status in (cc.COOT_EINVAL, cc.COOT_ESHAPE)
    with pytest.raises(cc.CootError) as e:
        coot.Batch([(X + b, None)])
    assert e.value.status == cc.COOT_EUNSUPPORTED


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_submatrix_views(coot, dtype):
    """submat / rows / cols / row / col: views with the parent's leading dimension, read in
    fused expressions and reductions and updated in place; the rest of the parent is
    left untouched (element by element against the oracle)."""
    g = synth.rng_for(93)
    P = synth.uniform(g, (150, 97), dtype)
    Q = synth.uniform(g, (150, 97), dtype)
    gP, gQ = coot.Mat.from_numpy(P, dtype=dtype), coot.Mat.from_numpy(Q, dtype=dtype)
    # Z-like expression over three views of P and Q (ragged 61 x 45 blocks, ld 150)
    sa, sb = gP.submat(5, 7, 65, 51), gQ.submat(80, 40, 140, 84)
    sc = gQ.submat(0, 0, 44, 60)                                # read through trans(): 45 x 61 -> 61 x 45
    got = coot.eval(2.0 * sa + sa % sb - coot.trans(sc)).numpy()
    A, B, C = P[5:66, 7:52], Q[80:141, 40:85], Q[0:45, 0:61]
    want = ew.evaluate([("scalar", 0), ("load", 0), ("schur",), ("load", 0), ("load", 1), ("schur",), ("add",),
                        ("load", 2), ("trans",), ("sub",)], [A, B, C], [2.0], dtype)
    assert np.array_equal(got, want)
    # reductions over a view
    s0 = coot.sum(sa, 0).numpy().ravel()
    for j in range(45):
        assert rd.rel_err(float(s0[j]), rd.exact_sum(A[:, j]), rd.sum_abs(A[:, j])) <= REL[dtype]
    v1 = coot.var(sa, dim=1).numpy().ravel()
    for i, q in enumerate(rd.var_dim(A, 1, dtype)):
        assert rd.rel_err(float(v1[i]), q, 1.0) <= REL[dtype]
    # rows, cols, a row (elements ld apart) and a column
    assert np.array_equal(coot.eval(gP.rows(10, 12) * 3.0).numpy(), P[10:13] * np.asarray(3.0, P.dtype))
    assert np.array_equal(coot.eval(gP.cols(90, 96) - gQ.cols(0, 6)).numpy(), P[:, 90:97] - Q[:, 0:7])
    r = gP.row(149)
    assert (r.n_rows, r.n_cols, r.ld) == (1, 97, 150)
    assert np.array_equal(coot.eval(r + gQ.row(0)).numpy(), (P[149] + Q[0]).reshape(1, -1))
    assert np.array_equal(coot.eval(gP.col(96) % gQ.col(1)).numpy(), (P[:, 96] * Q[:, 1]).reshape(-1, 1))
    # in-place update of a block (Armadillo's X.submat(...) += Y): only the block changes
    blk = gP.submat(100, 20, 149, 60)
    blk += 0.5 * gQ.submat(0, 0, 49, 40)
    expect = P.copy()
    expect[100:150, 20:61] = ew.evaluate([("load", 0), ("scalar", 0), ("load", 1), ("schur",), ("add",)],
                                         [P[100:150, 20:61], Q[0:50, 0:41]], [0.5], dtype)
    assert np.array_equal(gP.numpy(), expect)
    with pytest.raises(IndexError):
        gP.submat(0, 0, 150, 3)
