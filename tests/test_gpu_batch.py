"""Batched evaluation (one persistent, graph-captured launch) against the oracle and
against the single-expression fused path."""
import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from tests.exact import ulp_distance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def coot():
    import torch
    import paper_2508_11385_amd as coot
    coot.init(0)
    torch.cuda.synchronize()
    return coot


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


def _make(coot, n, seed, dtype="f32", lo=8, hi=128, depth_hi=6):
    g = synth.rng_for(seed)
    specs = synth.batch_workload(n, seed=seed, dtype=dtype, dim_lo=lo, dim_hi=hi, depth_hi=depth_hi)
    host, exprs = [], []
    for spec in specs:
        ops = synth.operands_for(spec, g)
        mats = [coot.Mat.from_numpy(o) for o in ops]
        host.append(ops)
        exprs.append(_build(coot, spec, mats))
    return specs, host, exprs


def _check_against_oracle(specs, host, outs, dtype):
    for spec, ops, out in zip(specs, host, outs):
        want = ew.evaluate(spec.postfix, ops, spec.scalars, dtype)
        got = out.numpy()
        d = ulp_distance(got, want)
        limit = 1 if any(p[0] == "exp" for p in spec.postfix) else 0
        assert np.max(d) <= limit, (spec.postfix, spec.out_shape, float(np.max(d)))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_matches_oracle_and_fused(coot, dtype):
    import torch
    specs, host, exprs = _make(coot, 120, 41 if dtype == "f32" else 42, dtype)
    b = coot.Batch([(e, None) for e in exprs])
    b.launch()
    torch.cuda.synchronize()
    _check_against_oracle(specs, host, b.outs, dtype)
    for e, out in zip(exprs[:40], b.outs[:40]):
        single = coot.eval(e).numpy()
        assert np.array_equal(np.ascontiguousarray(single).view(np.uint8),
                              np.ascontiguousarray(out.numpy()).view(np.uint8))   # bitwise, signed zeros too
    info = b.info()
    assert info["n_exprs"] == 120 and info["n_tiles"] > 120


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("cfg", [(4, 1, 2, 8), (4, 1, 1, 4, 32, 32)])
def test_multi_element_threads_match_oracle_and_fused(coot, dtype, cfg):
    """32 x 32 tiles by two wavefronts (8 elements per thread) and by one (16 per thread,
    transposed leaves staged by LDS DMA): every output against the oracle and bitwise
    against the single-expression fused path."""
    import torch
    specs, host, exprs = _make(coot, 80, 43 if dtype == "f32" else 44, dtype)
    b = coot.Batch([(e, None) for e in exprs], cfg=cfg)
    info = b.info()
    assert (info["tile"], info["g"], info["tile_2d"], info["g_2d"]) == (32, 4 // cfg[2], 32, 4 // cfg[2])
    b.launch()
    torch.cuda.synchronize()
    _check_against_oracle(specs, host, b.outs, dtype)
    for e, out in zip(exprs[:30], b.outs[:30]):
        single = coot.eval(e).numpy()
        assert np.array_equal(np.ascontiguousarray(single).view(np.uint8),
                              np.ascontiguousarray(out.numpy()).view(np.uint8))


def test_graph_replays_with_eager_work_between(coot):
    import torch
    specs, host, exprs = _make(coot, 60, 43)
    b = coot.Batch([(e, None) for e in exprs])
    b.launch()
    torch.cuda.synchronize()
    ref = [o.numpy().copy() for o in b.outs]
    for rep in range(4):
        for o in b.outs:
            o.tensor.zero_()                      # eager work on the same stream between replays
        scratch = torch.randn(1 << 20, device="cuda").sum()
        b.launch()
        torch.cuda.synchronize()
        for r, o in zip(ref, b.outs):
            assert np.array_equal(r, o.numpy()), f"replay {rep} differs from the first launch"
        del scratch


def test_per_expression_launches_and_tuning_agree(coot):
    import torch
    specs, host, exprs = _make(coot, 80, 44)
    b = coot.Batch([(e, None) for e in exprs])
    b.launch()
    torch.cuda.synchronize()
    ref = [o.numpy().copy() for o in b.outs]
    for o in b.outs:
        o.tensor.zero_()
    b.launch_each()
    torch.cuda.synchronize()
    for r, o in zip(ref, b.outs):
        assert np.array_equal(r, o.numpy())
    cfg, us = b.tune()
    assert cfg[2] in (1, 2, 4) and cfg[0] in (1, 4) and us > 0
    for o in b.outs:
        o.tensor.zero_()
    b.launch()
    torch.cuda.synchronize()
    for r, o in zip(ref, b.outs):
        assert np.array_equal(r, o.numpy())


@pytest.mark.parametrize("cfg", [(1, 1, 1, 2), (4, 2, 4, 8), (4, 8, 1, 4), (1, 4, 4, 16),
                                 (4, 1, 2, 8), (1, 1, 2, 4), (4, 1, 1, 4, 32, 32), (1, 1, 1, 16, 32, 32)])
def test_every_tile_size_and_vector_width(coot, cfg):
    import torch
    specs, host, exprs = _make(coot, 40, 45, lo=1, hi=200)
    b = coot.Batch([(e, None) for e in exprs], cfg=cfg)
    b.launch()
    torch.cuda.synchronize()
    _check_against_oracle(specs, host, b.outs, "f32")


def test_many_transposed_leaves(coot):
    """Square operands read transposed: more transposed leaves than LDS slots go to global reads."""
    import torch
    g = synth.rng_for(46)
    n = 37
    mats_h = [synth.uniform(g, (n, n), "f32") for _ in range(6)]
    mats = [coot.Mat.from_numpy(m) for m in mats_h]
    e = coot.trans(mats[0]) + coot.trans(mats[1]) % coot.trans(mats[2]) - coot.trans(mats[3]) / \
        (1.0 + coot.abs(coot.trans(mats[4]))) + mats[5] % coot.trans(mats[5])
    post = coot.flatten(e).postfix
    want = ew.evaluate(post, mats_h, [1.0], "f32")
    # 6 transposed leaves: 4 LDS slots filled by LDS DMA on one-wave tiles (16 x 16, and
    # 32 x 32 with 16 elements per thread), 2 slots filled through registers on 32 x 32
    # tiles of two or four wavefronts; the rest read directly
    for cfg, slots in (((4, 4, 1, 4), 4), ((4, 4, 4, 4), 2), ((4, 4, 2, 4), 2), ((4, 4, 1, 4, 32, 32), 4)):
        b = coot.Batch([(e, None)], cfg=cfg)
        assert b.info()["lds_staged"] == slots
        b.launch()
        torch.cuda.synchronize()
        assert np.max(ulp_distance(b.outs[0].numpy(), want)) == 0, cfg


def test_batch_errors(coot):
    import paper_2508_11385_amd._coot as cc
    A = coot.Mat.from_numpy(np.ones((4, 4), np.uint32))
    with pytest.raises(cc.CootError) as e:
        coot.Batch([(A + A, None)])
    assert e.value.status == cc.COOT_EUNSUPPORTED
    S = coot.Mat.from_numpy(np.ones((5, 5), np.float32))
    with pytest.raises(cc.CootError) as e:
        coot.Batch([(coot.trans(S) + 1.0, S)])
    assert e.value.status == cc.COOT_EALIAS
    # an operand spanning 2 GiB or more (its two columns 2^29 floats apart): the interpreter's
    # 32-bit buffer offsets cannot reach it
    import torch
    big = torch.empty(2**29 + 64, dtype=torch.float32, device="cuda")
    W = coot.Mat(big.as_strided((4, 2), (1, 2**29)), "f32")
    with pytest.raises(cc.CootError) as e:
        coot.Batch([(W + 1.0, None)])
    assert e.value.status == cc.COOT_EUNSUPPORTED
    del W, big


def test_full_batch_workload_sampled(coot):
    """The 10,000-expression workload: every output computed in one launch, 300 checked in full."""
    import torch
    specs, host, exprs = _make(coot, 10_000, 3, lo=8, hi=512)
    b = coot.Batch([(e, None) for e in exprs])
    b.launch()
    torch.cuda.synchronize()
    pick = np.random.default_rng(9).choice(len(specs), 300, replace=False)
    _check_against_oracle([specs[i] for i in pick], [host[i] for i in pick], [b.outs[i] for i in pick], "f32")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_flat_chunks_unaligned_and_padded(coot, dtype):
    """Contiguous expressions run as flat chunks: ragged chunk tails, operands offset by one
    element (no 128-bit access), and a padded operand (falls back to 2-D tiles)."""
    import torch
    tdt = torch.float32 if dtype == "f32" else torch.float64
    g = synth.rng_for(47, 0 if dtype == "f32" else 1)
    exprs, want = [], []
    for k, (r, c) in enumerate([(1, 1), (3, 5), (33, 31), (257, 3), (1, 1031), (64, 64)]):
        hs = [synth.uniform(g, (r, c), dtype) for _ in range(3)]
        mats = []
        for j, h in enumerate(hs):
            if k % 2 == 1 and j == 1:            # offset view: misaligned storage
                base = torch.empty(r * c + 1, dtype=tdt, device="cuda")
                base[1:].copy_(torch.from_numpy(np.ascontiguousarray(h.T).ravel()))
                mats.append(coot.Mat(base[1:].view(c, r).t(), dtype))
            elif k == 5 and j == 2:              # leading dimension 67 > 64
                store = torch.zeros((c, r + 3), dtype=tdt, device="cuda")
                store[:, :r].copy_(torch.from_numpy(np.ascontiguousarray(h.T)))
                mats.append(coot.Mat(store[:, :r].t(), dtype))
            else:
                mats.append(coot.Mat.from_numpy(h))
        e = mats[0] % mats[1] - mats[2] / (1.0 + coot.abs(mats[0]))
        exprs.append(e)
        post = coot.flatten(e).postfix
        want.append(ew.evaluate(post, [hs[0], hs[1], hs[2]], [1.0], dtype))
    for cfg in (None, (4, 4, 1, 4), (1, 4, 4, 2), (4, 1, 2, 4), (4, 1, 1, 8, 32, 32), (1, 1, 1, 2, 32, 32)):
        b = coot.Batch([(e, None) for e in exprs], cfg=cfg)
        b.launch()
        torch.cuda.synchronize()
        for w, o in zip(want, b.outs):
            assert np.max(ulp_distance(o.numpy(), w)) == 0, cfg
