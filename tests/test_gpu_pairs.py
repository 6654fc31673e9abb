"""Two statements in one pass (out = e, then a full reduction of r over e's operands
and the result) against the same two statements run one after the other and the
oracle."""
import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from oracle import reduce as rd
from tests.exact import ulp_distance

pytestmark = pytest.mark.gpu

AXPY = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("add",)]


@pytest.fixture(scope="module")
def coot():
    import torch
    import paper_2508_11385_amd as coot
    coot.init(0)
    torch.cuda.synchronize()
    return coot


def test_axpy_then_dot_in_one_pass(coot):
    x, y = synth.axpy_inputs()
    gx, gy = coot.Mat.from_numpy(x, kind="col"), coot.Mat.from_numpy(y, kind="col")
    d = float(coot.eval_reduce(2.5 * gx + gy, gy, gx % gy).numpy()[0, 0])
    y_new = ew.evaluate(AXPY, [x, y], [2.5], "f32")
    assert np.max(ulp_distance(gy.numpy(), y_new)) == 0
    ref = rd.dot(x, y_new, "f32")
    assert rd.rel_err(d, ref, rd.to_float(rd.exact_dot(np.abs(x), np.abs(y_new)))) <= 1e-6
    # the same two statements one after the other
    gy2 = coot.Mat.from_numpy(y, kind="col")
    gy2 += 2.5 * gx
    d2 = float(coot.accu(gx % gy2).numpy()[0, 0])
    assert np.array_equal(gy2.numpy(), gy.numpy())
    assert rd.rel_err(d2, ref, 1.0) <= 1e-6


@pytest.mark.parametrize("dtype", ["f32", "f64", "f16"])
@pytest.mark.parametrize("kind", ["max", "min", "mean", "norm_inf", "norm1", "accu"])
def test_matrix_pairs(coot, dtype, kind):
    A, B, C, _ = synth.matrix_inputs(n_rows=300, n_cols=201, dtype=dtype)
    gA, gB, gC = (coot.Mat.from_numpy(m, dtype=dtype) for m in (A, B, C))
    out = coot.Mat.empty(300, 201, dtype)
    got = float(coot.eval_reduce(gA % gB + gC, out, (out - gA) * 0.5, kind).numpy()[0, 0])
    O = ew.evaluate([("load", 0), ("load", 1), ("schur",), ("load", 2), ("add",)], [A, B, C], [], dtype)
    assert np.array_equal(out.numpy(), O)
    Rv = ew.evaluate([("load", 0), ("load", 1), ("sub",), ("scalar", 0), ("schur",)], [O, A], [0.5], dtype)
    if kind in ("max", "min", "norm_inf"):
        want = {"max": rd.vmax, "min": rd.vmin, "norm_inf": rd.norm_inf}[kind](Rv, dtype)
        assert got == float(np.asarray(want, np.float64))
    else:
        exact = {"mean": rd.mean, "norm1": rd.norm1, "accu": rd.accu}[kind](Rv, dtype)
        if dtype == "f16":
            want = rd.round_exact(exact, dtype)
            assert abs(int(np.float16(got).view(np.int16)) - int(np.float16(want).view(np.int16))) <= 1
        else:
            scale = rd.sum_abs(Rv) / (Rv.size if kind == "mean" else 1)
            assert rd.rel_err(got, exact, scale) <= (1e-6 if dtype == "f32" else 1e-12)


def test_reads_before_the_store_through_the_operand_map(coot):
    """r_src naming the operand that out aliases reads the values as loaded (before the
    update); -1 reads the update."""
    import ctypes
    import paper_2508_11385_amd._coot as cc
    y = synth.uniform(synth.rng_for(95), (4096, 1), "f32")
    gy = coot.Mat.from_numpy(y, kind="col")
    he = coot.frontend.compiled(coot.flatten(gy + 1.0))
    hr = coot.frontend.compiled(coot.flatten(coot.Mat.from_numpy(y, kind="col") * 1.0))
    res = coot.Mat.empty(1, 1, "f32")
    cc.coot_expr_eval_reduce(he, [gy.operand()], [1.0], gy.operand(), hr, [0], [1.0], cc.COOT_RED_MAX,
                             res.operand(), None, coot.frontend._stream())
    assert float(res.numpy()[0, 0]) == float(y.max())                 # the old values
    cc.coot_expr_eval_reduce(he, [gy.operand()], [1.0], gy.operand(), hr, [-1], [1.0], cc.COOT_RED_MAX,
                             res.operand(), None, coot.frontend._stream())
    one = np.float32(1)
    assert float(res.numpy()[0, 0]) == float((np.float32(y.max()) + one) + one)  # y + 1, twice


def test_pair_errors(coot):
    import paper_2508_11385_amd._coot as cc
    A, B, C, D = synth.matrix_inputs(n_rows=40, n_cols=40)
    gA, gB, gD = coot.Mat.from_numpy(A), coot.Mat.from_numpy(B), coot.Mat.from_numpy(D)
    out = coot.Mat.empty(40, 40)
    with pytest.raises(cc.CootError) as e:                  # a transposed leaf needs the tiled kernels
        coot.eval_reduce(gA + coot.trans(gD), out, out + 0.0)
    assert e.value.status == cc.COOT_EUNSUPPORTED
    with pytest.raises(ValueError):                          # r may read only e's operands and out
        coot.eval_reduce(gA + 1.0, out, gB + out)
