"""coot_reduce_noalloc: the reduction entry point that allocates nothing (partial results
in the library's file-scope device scratch array) against coot_reduce, called through
the C ABI on the same inputs: bitwise equal, on two calls in a row, the second with a
smaller input; its refusals (kernels not loaded, partials beyond the array, the
unfused comparator); and a recording into a HIP graph replayed with eager work in
between."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2508_11385_amd as coot
    from paper_2508_11385_amd import _coot as cc
    from paper_2508_11385_amd import frontend as fe
    coot.init(0)
    torch.cuda.synchronize()
    return coot, cc, fe, torch


def _mats(coot, shapes, dtype, seed, dist="uniform"):
    g = synth.rng_for(77, seed)
    out = []
    for (r, c) in shapes:
        if dist == "lognormal":
            a = g.lognormal(0.0, 4.0, (r, c)) * g.choice([-1.0, 1.0], (r, c))
        else:
            a = g.uniform(-1, 1, (r, c))
        out.append(coot.Mat.from_numpy(a.astype(np.float32 if dtype != "f64" else np.float64), dtype))
    return out


def _z(coot, R, C, dtype, seed):
    A, B, Cm = _mats(coot, [(R, C)] * 3, dtype, seed)
    (D,) = _mats(coot, [(C, R)], dtype, seed + 100)
    return 2.0 * A + B % Cm - coot.trans(D)


def _out_shape(kind, dim, R, C, cc):
    if kind in (cc.COOT_RED_SUM, cc.COOT_RED_MEAN_DIM, cc.COOT_RED_VAR_DIM):
        return (1, C) if dim == 0 else (R, 1)
    return (1, 1)


def _both(env, e, kind, dim, flags=0):
    """coot_reduce and coot_reduce_noalloc of e into fresh outputs; their bytes."""
    coot, cc, fe, torch = env
    f = fe.flatten(e)
    h = fe.compiled(f)
    ops = [m.operand() for m in f.mats]
    R, C = cc.coot_expr_out_shape(h, ops)
    r, c = _out_shape(kind, dim, R, C, cc)
    outs = []
    for fn in (cc.coot_reduce, cc.coot_reduce_noalloc):
        o = coot.Mat.empty(r, c, f.dtype)
        o.tensor.fill_(float("nan"))
        fn(h, ops, f.scalars, kind, dim, flags, o.operand(), None, torch.cuda.current_stream().cuda_stream)
        outs.append(o)
    torch.cuda.synchronize()
    return [o.tensor.reshape(-1).contiguous().view(torch.uint8).cpu().numpy() for o in outs]


CASES = [
    ("sum0", "f32", lambda cc: (cc.COOT_RED_SUM, 0, 0)),
    ("sum1", "f32", lambda cc: (cc.COOT_RED_SUM, 1, 0)),
    ("var1", "f32", lambda cc: (cc.COOT_RED_VAR_DIM, 1, 0)),
    ("var0n", "f64", lambda cc: (cc.COOT_RED_VAR_DIM, 0, cc.COOT_RF_VAR_N)),
    ("mean1", "f16", lambda cc: (cc.COOT_RED_MEAN_DIM, 1, 0)),
    ("accu", "f32", lambda cc: (cc.COOT_RED_ACCU, -1, 0)),
    ("accu_plain", "f64", lambda cc: (cc.COOT_RED_ACCU, -1, cc.COOT_RF_PLAIN)),
    ("var", "f32", lambda cc: (cc.COOT_RED_VAR, -1, 0)),
    ("max", "bf16", lambda cc: (cc.COOT_RED_MAX, -1, 0)),
]


@pytest.mark.parametrize("name,dtype,spec", CASES, ids=[c[0] for c in CASES])
def test_tiled_reductions_equal_coot_reduce(env, name, dtype, spec):
    coot, cc, fe, torch = env
    kind, dim, flags = spec(cc)
    for k, (R, C) in enumerate([(1000, 700), (300, 257)]):       # the second call smaller
        a, b = _both(env, _z(coot, R, C, dtype, 10 * k + 1), kind, dim, flags)
        assert np.array_equal(a, b), f"{name} {R}x{C}: differs from coot_reduce"


def test_flat_dot_and_norm_equal_coot_reduce(env):
    coot, cc, fe, torch = env
    for k, n in enumerate([1_000_000, 1_000]):
        x, y = _mats(coot, [(n, 1), (n, 1)], "f32", 40 + k, "lognormal")
        for e, kind in ((x % y, cc.COOT_RED_ACCU), (x, cc.COOT_RED_NORM), (coot.abs(x), cc.COOT_RED_NORM1)):
            a, b = _both(env, e, kind, -1)
            assert np.array_equal(a, b), f"n={n} kind={kind}: differs from coot_reduce"


def test_norm_rescaling_path_equal_coot_reduce(env):
    """Squares that overflow binary32 take the rescaling kernels (their control word
    lives in the second half of the scratch)."""
    coot, cc, fe, torch = env
    for n in (70_000, 3):
        x = np.full((n, 1), 3e30, np.float32)
        x[1::2] = 4e30
        gx = coot.Mat.from_numpy(x, "f32", "col")
        a, b = _both(env, gx, cc.COOT_RED_NORM, -1)
        assert np.array_equal(a, b)
        assert np.isfinite(a.view(np.float32)).all()


def test_refusals(env):
    coot, cc, fe, torch = env
    s = torch.cuda.current_stream().cuda_stream
    # kernels never loaded for this expression: nothing compiled, nothing launched
    (x,) = _mats(coot, [(513, 3)], "f32", 90)
    f = fe.flatten(coot.sqrt(coot.abs(x)) - 0.125 * x)
    h = fe.compiled(f)
    o = coot.Mat.empty(1, 3, "f32")
    with pytest.raises(cc.CootError) as e:
        cc.coot_reduce_noalloc(h, [m.operand() for m in f.mats], f.scalars, cc.COOT_RED_SUM, 0, 0, o.operand(),
                               None, s)
    assert e.value.status == cc.COOT_EINVAL and "not loaded" in str(e.value)
    # partials beyond half of the array: a sum along dim 1 of a 2^21 x 1 column keeps
    # 2^21 float-float partials (16 MiB)
    (v,) = _mats(coot, [(1 << 21, 1)], "f32", 91)
    f = fe.flatten(v + v)
    h = fe.compiled(f)
    o = coot.Mat.empty(1 << 21, 1, "f32")
    ops = [m.operand() for m in f.mats]
    cc.coot_reduce(h, ops, f.scalars, cc.COOT_RED_SUM, 1, 0, o.operand(), None, s)   # loads the kernels
    with pytest.raises(cc.CootError) as e:
        cc.coot_reduce_noalloc(h, ops, f.scalars, cc.COOT_RED_SUM, 1, 0, o.operand(), None, s)
    assert e.value.status == cc.COOT_EUNSUPPORTED
    # the unfused comparator allocates temporaries
    f = fe.flatten(x + x)
    hu = fe.compiled(f, cc.COOT_CF_UNFUSED)
    o = coot.Mat.empty(1, 1, "f32")
    with pytest.raises(cc.CootError) as e:
        cc.coot_reduce_noalloc(hu, [m.operand() for m in f.mats], f.scalars, cc.COOT_RED_ACCU, -1, 0, o.operand(),
                               None, s)
    assert e.value.status == cc.COOT_EUNSUPPORTED
    torch.cuda.synchronize()


def test_recorded_into_a_graph(env):
    """The call recorded into a HIP graph (stream capture) and replayed, with eager
    reductions (through both entry points) between the replays, each replay equal to
    the eager result."""
    coot, cc, fe, torch = env
    e = _z(coot, 777, 513, "f32", 5)
    f = fe.flatten(e)
    h = fe.compiled(f)
    ops = [m.operand() for m in f.mats]
    ref = coot.Mat.empty(777, 1, "f32")
    cc.coot_reduce(h, ops, f.scalars, cc.COOT_RED_SUM, 1, 0, ref.operand(), None,
                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    want = ref.tensor.reshape(-1).contiguous().view(torch.uint8).cpu().numpy()
    out = coot.Mat.empty(777, 1, "f32")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cc.coot_reduce_noalloc(h, ops, f.scalars, cc.COOT_RED_SUM, 1, 0, out.operand(), None,
                               torch.cuda.current_stream().cuda_stream)
    other = _z(coot, 300, 257, "f32", 6)
    for rep in range(4):
        out.tensor.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        got = out.tensor.reshape(-1).contiguous().view(torch.uint8).cpu().numpy()
        assert np.array_equal(got, want), f"replay {rep} differs"
        a, b = _both(env, other, cc.COOT_RED_SUM, rep % 2)        # eager work on the same scratch
        assert np.array_equal(a, b)
    del g
