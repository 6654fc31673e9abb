"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: integers bit-exact; floating element-wise results within 1 ulp of
the per-operator rounded oracle (0 ulp expected for + - * / sqrt abs neg, trans);
fp32 reductions within 1e-6 relative error of the exact sum, fp64 within 1e-12.
"""
import gc
import math

import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from oracle import reduce as rd
from tests.exact import ulp_distance

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


def up(coot, a, kind=None):
    return coot.Mat.from_numpy(a, kind=kind)


def _z(coot, A, B, C, D):
    return 2.0 * A + B % C - coot.trans(D)


def _w(coot, A, B):
    return coot.exp(A) / (1.0 + coot.abs(B))


def _check_rel(got, exact_vals, scale_vals, tol, what):
    worst = 0.0
    for g, ref, sc in zip(got, exact_vals, scale_vals):
        e = rd.rel_err(float(g), ref, sc)
        worst = max(worst, e)
    assert worst <= tol, f"{what}: worst relative error {worst:.3e} > {tol:.0e}"
    return worst


SHAPES = [(1, 1), (3, 5), (64, 64), (67, 45), (130, 257), (256, 64), (1000, 3), (5, 1000)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", SHAPES)
def test_Z_and_W_elementwise(coot, dtype, shape):
    r, c = shape
    A, B, C, D = synth.matrix_inputs(n_rows=r, n_cols=c, dtype=dtype)
    gA, gB, gC, gD = (up(coot, x) for x in (A, B, C, D))
    Z = coot.eval(_z(coot, gA, gB, gC, gD)).numpy()
    W = coot.eval(_w(coot, gA, gB)).numpy()
    Zo = ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype)
    Wo = ew.evaluate(W_POST, [A, B], [1.0], dtype)
    assert Z.shape == Zo.shape == (r, c)
    assert np.max(ulp_distance(Z, Zo)) == 0, "Z uses only correctly rounded operators: 0 ulp expected"
    dW = ulp_distance(W, Wo)
    assert np.max(dW) <= 1, f"W: {int(np.sum(dW > 1))} elements beyond 1 ulp"


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(1, 1), (67, 45), (130, 257), (1000, 3), (3, 1000), (256, 128)])
def test_sum_dims_fused_and_materialised(coot, dtype, shape):
    r, c = shape
    A, B, C, D = synth.matrix_inputs(n_rows=r, n_cols=c, dtype=dtype)
    gA, gB, gC, gD = (up(coot, x) for x in (A, B, C, D))
    Zo = ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype)
    gZ = up(coot, Zo)
    for dim in (0, 1):
        ex = rd.sum_dim(Zo, dim, dtype)
        scale = [rd.sum_abs(v) for v in (Zo.T if dim == 0 else Zo)]
        fused = coot.sum(_z(coot, gA, gB, gC, gD), dim).numpy().ravel()
        mat = coot.sum(gZ, dim).numpy().ravel()
        assert fused.size == (c if dim == 0 else r)
        _check_rel(fused, ex, scale, REL[dtype], f"fused sum dim {dim}")
        _check_rel(mat, ex, scale, REL[dtype], f"materialised sum dim {dim}")


def test_axpy_then_dot_workload(coot):
    """y <- 2.5*x + y in place, then accu(x % y) with the updated y (n = 1,000,000)."""
    x, y = synth.axpy_inputs()
    gx, gy = up(coot, x, "col"), up(coot, y, "col")
    gy += 2.5 * gx
    y_new = ew.evaluate([("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("add",)], [x, y], [2.5], "f32")
    assert np.max(ulp_distance(gy.numpy(), y_new)) == 0
    got = float(coot.accu(gx % gy).numpy()[0, 0])
    ref = rd.dot(x, y_new, "f32")
    err = rd.rel_err(got, ref, rd.to_float(rd.exact_dot(np.abs(x), np.abs(y_new))))
    assert err <= 1e-6, err
    got_dot = float(coot.dot(gx, gy).numpy()[0, 0])
    assert got_dot == got
    plain = float(coot.accu(gx % gy, plain=True).numpy()[0, 0])
    assert rd.rel_err(plain, ref, 1.0) < 1e-3          # the comparator is merely less accurate


def test_contraction_is_off(coot):
    """2.5*x + y is rounded per operator on the device (no FMA contraction)."""
    x = np.full((256, 1), 0.1, np.float32)
    p = np.float32(np.float64(2.5) * np.float64(np.float32(0.1)))
    y = np.full((256, 1), np.float32(-p) + np.float32(2.0 ** -30), np.float32)
    gx, gy = up(coot, x, "col"), up(coot, y, "col")
    out = coot.eval(2.5 * gx + gy).numpy()
    want = ew.evaluate([("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("add",)], [x, y], [2.5], "f32")
    assert np.array_equal(out, want)


@pytest.mark.parametrize("shape", [(1000, 700), (67, 45), (8, 8)])
def test_integer_expressions(coot, shape):
    r, c = shape
    A, B, C = synth.int_inputs(which="u32", n_rows=r, n_cols=c)
    got = coot.eval((up(coot, A) + up(coot, B)) % up(coot, C)).numpy()
    want = ew.evaluate([("load", 0), ("load", 1), ("add",), ("load", 2), ("schur",)], [A, B, C], [], "u32")
    assert np.array_equal(got, want)
    for which in ("s32_full", "s32_small"):
        A, B = synth.int_inputs(which=which, n_rows=r, n_cols=c)
        got = coot.eval(up(coot, A) - 3 * up(coot, B)).numpy()
        want = ew.evaluate([("load", 0), ("scalar", 0), ("load", 1), ("schur",), ("sub",)], [A, B], [3.0], "s32")
        assert np.array_equal(got, want)
        # integer reductions wrap mod 2^32 and are bit-exact
        gA = up(coot, A)
        assert int(coot.accu(gA).numpy()[0, 0]) == rd.accu(A, "s32")
        assert [int(v) for v in coot.sum(gA, 0).numpy().ravel()] == rd.sum_dim(A, 0, "s32")
        assert [int(v) for v in coot.sum(gA, 1).numpy().ravel()] == rd.sum_dim(A, 1, "s32")


def test_accu_and_norm_lognormal(coot):
    x = synth.lognormal_signed(synth.rng_for(2, 9), 1 << 22).reshape(-1, 1)
    gx = up(coot, x, "col")
    s_ref = rd.accu(x, "f32")
    sc = rd.sum_abs(x)
    got = float(coot.accu(gx).numpy()[0, 0])
    assert rd.rel_err(got, s_ref, sc) <= 1e-6
    n_ref = rd.norm(x, "f32")
    got_n = float(coot.norm(gx).numpy()[0, 0])
    assert abs(got_n - n_ref) / n_ref <= 1e-6
    plain = float(coot.accu(gx, plain=True).numpy()[0, 0])
    print(f"\naccu rel err: compensated {rd.rel_err(got, s_ref, sc):.2e}, plain {rd.rel_err(plain, s_ref, sc):.2e}")


def test_norm_rescaling_and_closed_forms(coot):
    big = np.array([[3 * 2.0 ** 100], [4 * 2.0 ** 100]], np.float32)
    small = np.array([[3 * 2.0 ** -100], [4 * 2.0 ** -100]], np.float32)
    assert float(coot.norm(up(coot, big, "col")).numpy()[0, 0]) == 5 * 2.0 ** 100
    assert float(coot.norm(up(coot, small, "col")).numpy()[0, 0]) == 5 * 2.0 ** -100
    ones = up(coot, np.ones((1 << 20, 1), np.float32), "col")
    assert float(coot.accu(ones).numpy()[0, 0]) == float(1 << 20)
    v = np.concatenate([[np.float32(2 ** 24)], np.ones(1 << 20, np.float32)]).reshape(-1, 1)
    assert float(coot.accu(up(coot, v, "col")).numpy()[0, 0]) == 2 ** 24 + 2 ** 20
    x = synth.uniform(synth.rng_for(5, 5), (4096, 1), "f32")
    gx = up(coot, x, "col")
    nrm = float(coot.norm(gx).numpy()[0, 0])
    d = float(coot.dot(gx, gx).numpy()[0, 0])
    assert abs(nrm * nrm - d) / d < 1e-6


def _tree_case(coot, spec, ops, dtype):
    got = coot.eval(_build(coot, spec, [up(coot, o) for o in ops])).numpy()
    want = ew.evaluate(spec.postfix, ops, spec.scalars, dtype)
    return got, want


def _build(coot, spec, mats):
    st = []
    for it in spec.postfix:
        op = it[0]
        if op == "load":
            st.append(mats[it[1]])
        elif op == "scalar":
            st.append(coot.Scalar(spec.scalars[it[1]]))
        elif op in ("add", "sub", "schur", "div"):
            b, a = st.pop(), st.pop()
            st.append(coot.Node(op, [a, b]))
        else:
            st.append(coot.Node(op, [st.pop()]))
    return st[0]


@pytest.mark.parametrize("dtype", ["f32", "f64", "u32", "s32"])
def test_random_trees(coot, dtype):
    g = synth.rng_for(123, {"f32": 0, "u32": 1, "s32": 2, "f64": 3}[dtype])
    n_exp_1ulp = 0
    for trial in range(60):
        r, c = int(g.integers(1, 150)), int(g.integers(1, 150))
        spec = synth.random_tree(g, int(g.integers(1, 7)), int(g.integers(2, 6)), r, c, dtype)
        ops = synth.operands_for(spec, g)
        got, want = _tree_case(coot, spec, ops, dtype)
        if dtype in ("f32", "f64"):
            d = ulp_distance(got, want)
            has_exp = any(p[0] == "exp" for p in spec.postfix)
            limit = 1 if has_exp else 0
            assert np.max(d) <= limit, (spec.postfix, r, c, np.max(d))
            n_exp_1ulp += int(np.sum(d == 1))
        else:
            assert np.array_equal(got, want), spec.postfix


def test_fused_equals_unfused_bitwise(coot):
    A, B, C, D = synth.matrix_inputs(n_rows=300, n_cols=170)
    gA, gB, gC, gD = (up(coot, x) for x in (A, B, C, D))
    for e in (_z(coot, gA, gB, gC, gD), _w(coot, gA, gB)):
        f = coot.eval(e).numpy()
        u = coot.eval(e, unfused=True).numpy()
        assert np.array_equal(f.view(np.uint32), u.view(np.uint32))
    s_f = coot.sum(_z(coot, gA, gB, gC, gD), 1).numpy()
    s_u = coot.sum(_z(coot, gA, gB, gC, gD), 1, unfused=True).numpy()
    assert np.array_equal(s_f, s_u)


def test_determinism(coot):
    x = synth.lognormal_signed(synth.rng_for(2, 10), 3_000_001).reshape(-1, 1)
    gx = up(coot, x, "col")
    a = [coot.accu(gx).numpy()[0, 0] for _ in range(3)]
    assert a[0] == a[1] == a[2]
    A, B, C, D = synth.matrix_inputs(n_rows=513, n_cols=257)
    gs = [up(coot, m) for m in (A, B, C, D)]
    s = [coot.sum(_z(coot, *gs), 1).numpy() for _ in range(2)]
    assert np.array_equal(s[0], s[1])


def test_dim_sums_many_partials_and_repeats(coot):
    """Tall and wide operands give hundreds of segment partials per output; calls of
    different shapes alternate and repeat and must give identical bits each time."""
    g = synth.rng_for(2, 11)
    T = synth.uniform(g, (20000, 130), "f32")
    Wd = synth.uniform(g, (130, 20000), "f32")
    S = synth.uniform(g, (67, 45), "f32")
    gT, gW, gS = up(coot, T), up(coot, Wd), up(coot, S)
    calls = [(gT, 0), (gW, 1), (gS, 0), (gT, 1), (gW, 0), (gS, 1)]
    first = [coot.sum(m, d).numpy().ravel() for m, d in calls]
    for _ in range(2):
        again = [coot.sum(m, d).numpy().ravel() for m, d in calls]
        assert all(np.array_equal(a, b) for a, b in zip(first, again))
    for (m, d), got in zip(calls, first):
        h = {id(gT): T, id(gW): Wd, id(gS): S}[id(m)]
        ex = rd.sum_dim(h, d, "f32")
        scale = [rd.sum_abs(v) for v in (h.T if d == 0 else h)]
        _check_rel(got, ex, scale, REL["f32"], f"sum dim {d} of {h.shape}")


def test_edge_cases(coot):
    import paper_2508_11385_amd._coot as cc
    E = up(coot, np.zeros((0, 5), np.float32))
    assert coot.eval(E + 1.0).numpy().shape == (0, 5)
    assert float(coot.accu(E).numpy()[0, 0]) == 0.0
    assert np.all(coot.sum(E, 0).numpy() == 0)
    A = up(coot, np.ones((4, 6), np.float32))
    B = up(coot, np.ones((6, 4), np.float32))
    with pytest.raises(cc.CootError) as e:
        coot.eval(A + B)
    assert e.value.status == cc.COOT_ESHAPE
    S = up(coot, np.ones((5, 5), np.float32))
    with pytest.raises(cc.CootError) as e:
        coot.eval(coot.trans(S) + 1.0, out=S)       # reads S transposed while writing it
    assert e.value.status == cc.COOT_EALIAS
    with pytest.raises(cc.CootError) as e:
        coot.eval(A + A, out=coot.Mat.empty(6, 4))
    assert e.value.status == cc.COOT_ESHAPE
    # a strided (submatrix-like) operand goes through the tiled path
    import torch
    big = torch.arange(40 * 30, dtype=torch.float32, device="cuda").reshape(30, 40).t()   # 40 x 30, ld 40
    sub = coot.Mat(big[:33, :], "f32")                                                   # 33 x 30, ld 40
    got = coot.eval(sub * 2.0).numpy()
    want = big[:33, :].cpu().numpy() * 2
    assert np.array_equal(got, want)


# ---------------------------------------------------------------------------
# Full-size workloads: sampled outputs the oracle computes one by one, plus
# properties that hold at any size.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_full_size_matrix_workload(coot, dtype):
    A, B, C, D = synth.matrix_inputs(4096, dtype)
    gA, gB, gC, gD = (up(coot, x) for x in (A, B, C, D))
    Zg = coot.eval(_z(coot, gA, gB, gC, gD))
    Wg = coot.eval(_w(coot, gA, gB))
    g = np.random.default_rng(7)
    rows = g.integers(0, 4096, 50_000)
    cols = g.integers(0, 4096, 50_000)
    Z = Zg.numpy()
    W = Wg.numpy()
    zo = ew.evaluate_at(Z_POST, [A, B, C, D], [2.0], dtype, rows, cols)
    wo = ew.evaluate_at(W_POST, [A, B], [1.0], dtype, rows, cols)
    assert np.max(ulp_distance(Z[rows, cols], zo)) == 0
    assert np.max(ulp_distance(W[rows, cols], wo)) <= 1
    s0 = coot.sum(_z(coot, gA, gB, gC, gD), 0).numpy().ravel()
    s1 = coot.sum(_z(coot, gA, gB, gC, gD), 1).numpy().ravel()
    jj = g.integers(0, 4096, 24)
    ii = g.integers(0, 4096, 24)
    for j in jj:
        col = ew.evaluate_at(Z_POST, [A, B, C, D], [2.0], dtype, np.arange(4096), np.full(4096, j))
        assert rd.rel_err(float(s0[j]), rd.exact_sum(col), rd.sum_abs(col)) <= REL[dtype]
    for i in ii:
        row = ew.evaluate_at(Z_POST, [A, B, C, D], [2.0], dtype, np.full(4096, i), np.arange(4096))
        assert rd.rel_err(float(s1[i]), rd.exact_sum(row), rd.sum_abs(row)) <= REL[dtype]


@pytest.mark.parametrize("dtype,shape", [("f32", (8192, 8192)), ("f64", (4096, 4200))])
def test_flat_evaluation_beyond_the_infinity_cache(coot, dtype, shape):
    """W over operands larger than 256 MiB together (512 MiB fp32, 262.5 MiB fp64): the
    flat kernel then loads them non-temporally; sampled outputs against the oracle,
    and a misaligned view of the same data (the one-element fallback kernel)."""
    import torch
    R, C = shape
    g = synth.rng_for(49, 0 if dtype == "f32" else 1)
    A = synth.uniform(g, (R, C), dtype)
    B = synth.uniform(g, (R, C), dtype)
    gA, gB = up(coot, A), up(coot, B)
    W = coot.eval(_w(coot, gA, gB)).numpy()
    r = np.random.default_rng(3)
    rows, cols = r.integers(0, R, 50_000), r.integers(0, C, 50_000)
    wo = ew.evaluate_at(W_POST, [A, B], [1.0], dtype, rows, cols)
    assert np.max(ulp_distance(W[rows, cols], wo)) <= 1
    del W
    # the same values one element off a 16-byte boundary
    tdt = torch.float32 if dtype == "f32" else torch.float64
    base = torch.empty(R * C + 1, dtype=tdt, device="cuda")
    base[1:].copy_(gA.tensor.t().reshape(-1))
    mA = coot.Mat(base[1:].view(C, R).t(), dtype)
    W1 = coot.eval(_w(coot, mA, gB)).numpy()
    assert np.max(ulp_distance(W1[rows, cols], wo)) <= 1


FLAT_CFGS = [(2, 8, 4, 16), (4, 8, 8, 2), (1, 8, 1, 16), (4, 2, 4, 4), (2, 4, 8, 16), (1, 1, 4, 4),
             (4, 1, 4, 2), (2, 2, 2, 8)]


@pytest.mark.parametrize("dtype", ["f32", "f64", "u32"])
def test_flat_launch_settings_match_oracle(coot, dtype):
    """Flat evaluation on a ragged 1000 x 333 shape under a spread of launch settings
    (vector width, groups per thread per trip, waves, workgroups per CU), the element-wise
    default past 2^24 elements first: every element against the oracle (0 ulp, and at
    most 1 ulp where exp appears)."""
    R, C = 1000, 333
    if dtype == "u32":
        A, B, Cm = synth.int_inputs(which="u32", n_rows=R, n_cols=C)
        gA, gB, gC = up(coot, A), up(coot, B), up(coot, Cm)
        exprs = [((gA + gB) % gC, [A, B, Cm], 0)]
    else:
        A, B, Cm, _ = synth.matrix_inputs(dtype=dtype, n_rows=R, n_cols=C)
        gA, gB, gC = up(coot, A), up(coot, B), up(coot, Cm)
        exprs = [(2.0 * gA + gB % gC - gA, [A, B, Cm], 0), (_w(coot, gA, gB), [A, B], 1)]
    for e, leaves, tol in exprs:
        flat = coot.flatten(e)
        src = {id(gA): A, id(gB): B, id(gC): Cm}
        assert [src[id(m)] is l for m, l in zip(flat.mats, leaves)] == [True] * len(leaves)
        want = ew.evaluate(flat.postfix, leaves, flat.scalars, dtype)
        for cfg in FLAT_CFGS:
            got = coot.eval(e, cfg=cfg).numpy()
            if tol == 0:
                assert got.dtype == want.dtype and np.array_equal(
                    np.ascontiguousarray(got).view(np.uint8), np.ascontiguousarray(want).view(np.uint8)), (dtype, cfg)
            else:
                assert np.max(ulp_distance(got, want)) <= tol, (dtype, cfg)


def test_full_size_integer_workload(coot):
    A, B, C = synth.int_inputs(8192, "u32")
    got = coot.eval((up(coot, A) + up(coot, B)) % up(coot, C)).numpy()
    g = np.random.default_rng(8)
    rows, cols = g.integers(0, 8192, 100_000), g.integers(0, 8192, 100_000)
    post = [("load", 0), ("load", 1), ("add",), ("load", 2), ("schur",)]
    assert np.array_equal(got[rows, cols], ew.evaluate_at(post, [A, B, C], [], "u32", rows, cols))
    del got
    for which in ("s32_full", "s32_small"):
        A, B = synth.int_inputs(8192, which)
        got = coot.eval(up(coot, A) - 3 * up(coot, B)).numpy()
        post = [("load", 0), ("scalar", 0), ("load", 1), ("schur",), ("sub",)]
        assert np.array_equal(got[rows, cols], ew.evaluate_at(post, [A, B], [3.0], "s32", rows, cols))


def test_full_size_hard_reductions(coot):
    x = synth.hard_reduction_inputs()
    gx = up(coot, x, "col")
    got = float(coot.accu(gx).numpy()[0, 0])
    got_n = float(coot.norm(gx).numpy()[0, 0])
    plain = float(coot.accu(gx, plain=True).numpy()[0, 0])
    plain_n = float(coot.norm(gx, plain=True).numpy()[0, 0])
    ref = rd.accu(x, "f32")
    sc = rd.sum_abs(x)
    nref = rd.norm(x, "f32")
    e_acc = rd.rel_err(got, ref, sc)
    e_nrm = abs(got_n - nref) / nref
    print(f"\n2^28 lognormal: accu rel err {e_acc:.2e} (plain {rd.rel_err(plain, ref, sc):.2e}), "
          f"norm rel err {e_nrm:.2e} (plain {abs(plain_n - nref) / nref:.2e}), "
          f"kappa {sc / abs(float(ref)):.2f}")
    assert e_acc <= 1e-6 and e_nrm <= 1e-6


def test_caller_allocator_for_workspaces_and_temporaries(coot):
    """Workspaces and comparator temporaries come from PyTorch's caching allocator while it
    is installed, results are bitwise those of hipMalloc'd buffers, and switching back
    hands every buffer to the allocator that provided it."""
    import torch
    import paper_2508_11385_amd._coot as cc
    A, B, C, D = synth.matrix_inputs(n_rows=300, n_cols=200)
    gs = [up(coot, m) for m in (A, B, C, D)]
    flat = coot.flatten(_z(coot, *gs))
    h = coot.frontend.compiled(flat)
    hu = coot.frontend.compiled(flat, cc.COOT_CF_UNFUSED)
    ops = [m.operand() for m in flat.mats]
    stream = torch.cuda.current_stream().cuda_stream

    def run():
        s0, u = coot.Mat.empty(1, 200, "f32", "row"), coot.Mat.empty(300, 200)
        cc.coot_reduce(h, ops, flat.scalars, cc.COOT_RED_SUM, 0, 0, s0.operand(), None, stream)
        cc.coot_expr_eval(hu, ops, flat.scalars, u.operand(), None, stream)
        torch.cuda.synchronize()
        return s0.numpy(), u.numpy()

    ref = run()
    gc.collect()                                 # nothing of earlier tests is freed while measuring
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    coot.use_torch_allocator(True)
    try:
        got = run()
        during = torch.cuda.memory_allocated()
    finally:
        coot.use_torch_allocator(False)
    # the library holds at least one 64 KiB workspace from the caching allocator, and
    # hands it back when the allocator is switched off
    assert during - base >= 65536, "no library buffer came from the caching allocator"
    assert during - torch.cuda.memory_allocated() >= 65536
    assert all(np.array_equal(a, b) for a, b in zip(ref, got))
    assert all(np.array_equal(a, b) for a, b in zip(ref, run()))


TILES = [(64, 64), (128, 32), (32, 128), (256, 16), (16, 256), (128, 64), (32, 32), (64, 16), (16, 64), (128, 8),
         (256, 8), (128, 16), (64, 32)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("tile", TILES)
def test_tile_shapes(coot, dtype, tile):
    """Every tile shape of the tiled kernels, through element-wise evaluation, full and
    dimension reductions, on a ragged shape (partial tiles on both edges) and an aligned
    one with 4-element groups: Z 0 ulp, sums within the reduction tolerance, max exact."""
    import paper_2508_11385_amd._coot as cc
    for (r, c), vec in (((300, 170), 1), ((512, 256), 4 if dtype == "f32" else 2)):
        cfg = (vec, 0, 0, 0) + tile
        A, B, C, D = synth.matrix_inputs(n_rows=r, n_cols=c, dtype=dtype)
        gA, gB, gC, gD = (up(coot, x) for x in (A, B, C, D))
        if tile[0] * (tile[1] + 1) * (8 if dtype == "f64" else 4) > 65536:
            # the staged transposed leaf of D does not fit 64 KiB of LDS: refused, nothing launched
            with pytest.raises(cc.CootError) as ei:
                coot.eval(_z(coot, gA, gB, gC, gD), cfg=cfg)
            assert ei.value.status == cc.COOT_EINVAL and "64 KiB" in str(ei.value)
            continue
        Zo = ew.evaluate(Z_POST, [A, B, C, D], [2.0], dtype)
        Z = coot.eval(_z(coot, gA, gB, gC, gD), cfg=cfg).numpy()
        assert np.max(ulp_distance(Z, Zo)) == 0, (tile, r, c)
        for dim in (0, 1):
            got = coot.sum(_z(coot, gA, gB, gC, gD), dim, cfg=cfg).numpy().ravel()
            scale = [rd.sum_abs(v) for v in (Zo.T if dim == 0 else Zo)]
            _check_rel(got, rd.sum_dim(Zo, dim, dtype), scale, REL[dtype], f"sum dim {dim} {tile}")
        got = float(coot.accu(_z(coot, gA, gB, gC, gD), cfg=cfg).numpy()[0, 0])
        assert rd.rel_err(got, rd.accu(Zo, dtype), rd.sum_abs(Zo)) <= REL[dtype], tile
        assert float(coot.max(_z(coot, gA, gB, gC, gD), cfg=cfg).numpy()[0, 0]) == float(np.max(Zo))
        v1 = coot.var(_z(coot, gA, gB, gC, gD), dim=1, cfg=cfg).numpy().ravel()
        want = rd.var_dim(Zo, 1, dtype, 0)
        for gv, q in zip(v1, want):
            assert rd.rel_err(float(gv), q, abs(float(q))) <= REL[dtype], tile
