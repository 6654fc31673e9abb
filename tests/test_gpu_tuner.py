"""The learned tuner on the GPU: MLP forward / gradients / Adam against the binary64
oracle, training, the autotuner's timing table and its policies."""
import math

import numpy as np
import pytest

import synth
from oracle import mlp as om
from oracle import elementwise as ew

pytestmark = pytest.mark.gpu

F, H1, H2 = 17, 64, 64


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2508_11385_amd as coot
    from paper_2508_11385_amd import _coot as cc
    coot.init(0)
    torch.cuda.synchronize()
    return coot, cc, torch


def _init_params(seed, f=F, h1=H1, h2=H2):
    """He-initialised weights drawn on the host (the random numbers are inputs to both sides)."""
    g = synth.rng_for(40, seed)
    p = {"W1": g.normal(0, math.sqrt(2 / f), (h1, f)), "b1": g.normal(0, 0.05, h1),
         "W2": g.normal(0, math.sqrt(2 / h1), (h2, h1)), "b2": g.normal(0, 0.05, h2),
         "W3": g.normal(0, math.sqrt(2 / h2), (1, h2)), "b3": g.normal(0, 0.05, 1)}
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    flat = np.concatenate([p[k].ravel() for k in om.PARAM_ORDER]).astype(np.float32)
    return p, flat


def _unflat(flat, f=F, h1=H1, h2=H2):
    shapes = {"W1": (h1, f), "b1": (h1,), "W2": (h2, h1), "b2": (h2,), "W3": (1, h2), "b3": (1,)}
    out, o = {}, 0
    for k in om.PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = flat[o:o + n].reshape(shapes[k]).astype(np.float64)
        o += n
    return out


def _batch(seed, B):
    g = synth.rng_for(41, seed)
    X = g.normal(size=(B, F)).astype(np.float32)
    y = g.normal(size=B).astype(np.float32)
    mask = (g.uniform(size=B) < 0.85).astype(np.float32)
    return X, y, mask


def test_forward_and_gradients_match_oracle(env):
    coot, cc, torch = env
    p, flat = _init_params(1)
    X, y, mask = _batch(1, 96)
    m = cc.coot_mlp_create(F, H1, H2, flat)
    dX, dy, dm = (torch.from_numpy(a).cuda() for a in (X, y, mask))
    out = torch.empty(96, device="cuda")
    loss = torch.empty(1, device="cuda")
    cc.coot_mlp_forward(m, dX.data_ptr(), 96, out.data_ptr())
    ref_out, cache = om.forward(p, X.astype(np.float64))
    assert np.allclose(out.cpu().numpy(), ref_out, rtol=1e-5, atol=1e-5)
    inv = 1.0 / float(mask.sum())
    cc.coot_mlp_backward(m, dX.data_ptr(), dy.data_ptr(), dm.data_ptr(), 96, inv, loss.data_ptr())
    torch.cuda.synchronize()
    assert abs(loss.item() - om.loss(ref_out, y, mask)) <= 1e-5 * max(1.0, om.loss(ref_out, y, mask))
    g = _unflat(cc.coot_mlp_get_grads(m))
    ref = om.backward(p, cache, ref_out, y.astype(np.float64), mask.astype(np.float64))
    for k in om.PARAM_ORDER:
        err = np.linalg.norm(g[k] - ref[k]) / max(np.linalg.norm(ref[k]), 1e-30)
        assert err <= 1e-4, (k, err)
    cc.coot_mlp_release(m)


def test_adam_step_matches_oracle(env):
    coot, cc, torch = env
    p, flat = _init_params(2)
    X, y, mask = _batch(2, 64)
    m = cc.coot_mlp_create(F, H1, H2, flat)
    dX, dy, dm = (torch.from_numpy(a).cuda() for a in (X, y, mask))
    inv = 1.0 / float(mask.sum())
    pp = {k: v.copy() for k, v in p.items()}
    mom, vel = om.zeros_like(pp), om.zeros_like(pp)
    for t in (1, 2, 3):
        cc.coot_mlp_backward(m, dX.data_ptr(), dy.data_ptr(), dm.data_ptr(), 64, inv)
        cc.coot_mlp_adam_step(m, 1e-3, 0.9, 0.999, 1e-8, t)
        out, cache = om.forward(pp, X.astype(np.float64))
        gr = om.backward(pp, cache, out, y.astype(np.float64), mask.astype(np.float64))
        pp, mom, vel = om.adam_step(pp, gr, mom, vel, t)
    got = _unflat(cc.coot_mlp_get_params(m))
    for k in om.PARAM_ORDER:
        # each Adam step moves a parameter by about lr; fp32 vs fp64 differ far below that
        assert np.max(np.abs(got[k] - pp[k])) <= 2e-5, k
    cc.coot_mlp_release(m)


def test_training_reduces_loss(env):
    coot, cc, torch = env
    _, flat = _init_params(3)
    g = synth.rng_for(42)
    X = g.normal(size=(2048, F)).astype(np.float32)
    w = g.normal(size=F)
    y = (np.tanh(X @ w * 0.3) + 0.1 * X[:, 0] ** 2).astype(np.float32)
    mask = np.ones(2048, np.float32)
    m = cc.coot_mlp_create(F, H1, H2, flat)
    dX, dy, dm = (torch.from_numpy(a).cuda() for a in (X, y, mask))
    losses = cc.coot_mlp_train(m, dX.data_ptr(), dy.data_ptr(), dm.data_ptr(), mask, 2048, 256, 40, 7, 3e-3)
    assert losses[-1] < 0.2 * losses[0], losses
    cc.coot_mlp_release(m)


def test_tune_table_and_policies(env):
    coot, cc, torch = env
    A, B, C, D = synth.matrix_inputs(n_rows=1000, n_cols=300)
    gA, gB = coot.Mat.from_numpy(A), coot.Mat.from_numpy(B)
    e = coot.exp(gA) / (1.0 + coot.abs(gB))
    flat = coot.flatten(e)
    h = coot.frontend.compiled(flat)
    ops = [m_.operand() for m_ in flat.mats]
    out = coot.Mat.empty(1000, 300)
    fam = cc.coot_tune_prepare(h, ops, -1)
    space = cc.coot_tune_space(fam)
    t = cc.coot_tune_table(h, ops, flat.scalars, out.operand(), -1, space, reps=3, flush=True)
    assert len(t) == len(space) and all(x > 0 for x in t if not math.isnan(x))
    want = ew.evaluate(flat.postfix, [A, B], flat.scalars, "f32")
    for cfg in (space[0], space[len(space) // 2], space[-1]):
        out.tensor.zero_()
        cc.coot_tune_launch(h, ops, flat.scalars, out.operand(), -1, cfg)
        torch.cuda.synchronize()
        assert np.array_equal(out.numpy(), want)
    best, us = cc.coot_tune(h, ops, flat.scalars, out.operand(), -1, 1)
    assert best in space and us > 0
    dflt, us_d = cc.coot_tune(h, ops, flat.scalars, out.operand(), -1, 0)
    assert us <= us_d * 1.5
    # accu through the tuning module matches the fused reduction
    hx = coot.frontend.compiled(coot.flatten(gA % gB))
    acc = coot.Mat.empty(1, 1)
    cc.coot_tune_launch(hx, [gA.operand(), gB.operand()], [], acc.operand(), 0, (4, 4, 4, 8))
    ref = coot.accu(gA % gB).numpy()[0, 0]
    torch.cuda.synchronize()
    assert acc.numpy()[0, 0] == ref


def test_costmodel_roundtrip_and_prediction(env, tmp_path):
    coot, cc, torch = env
    NF = cc.N_FEATURES
    flat = np.concatenate([_init_params(4 + k, f=NF)[1] for k in range(3)])   # an ensemble of 3
    g = synth.rng_for(43)
    X = g.normal(size=(512, NF)).astype(np.float32)
    y = (X[:, 6] + 0.5 * X[:, 13]).astype(np.float32)     # depends on rows and vec
    mask = np.ones(512, np.float32)
    cm, losses = cc.coot_costmodel_train(X, y, mask, flat, H1, H2, 30, 128, 5, 3e-3, n_models=3)
    assert losses[-1] < losses[0]
    h = cc.coot_expr_compile([("load", 0), ("load", 1), ("add",)], [(cc.COOT_F32, 0)] * 2, 0)
    space = cc.coot_tune_space(0)
    best, pred = cc.coot_costmodel_predict(cm, h, 4096, 4096, 0, space)
    assert 0 <= best < len(space) and np.all(pred > 0) and pred[best] == pred.min()
    path = str(tmp_path / "cm.bin")
    cc.coot_costmodel_save(cm, path)
    cm2 = cc.coot_costmodel_load(path)
    best2, pred2 = cc.coot_costmodel_predict(cm2, h, 4096, 4096, 0, space)
    assert best2 == best and np.array_equal(pred, pred2)
    cc.coot_costmodel_release(cm)
    cc.coot_costmodel_release(cm2)


def test_trained_cost_model_against_the_default(env):
    """The learned part against the method without it: on held-out signatures, the
    library's cost-model policy (the trained ensemble's argmin where it predicts at least
    5 % over the library default, else the default) and the default configuration, both
    scored by regret within one exhaustive timing table built here (t(pick) / t(table's
    best) - 1: the same table for both, so no re-timing noise enters the comparison).
    The default is itself the fixed configuration fastest over the autotuner's tables,
    so on these small signatures (outputs up to 4096 x 4096) the two are close: the policy
    must not lose more than 1.5 points to the default and must stay within 12 % of
    exhaustive autotuning; and the trained network's plain argmin must beat an untrained
    network's by a fifth (training on 160 signatures' tables ranks configurations)."""
    coot, cc, torch = env
    from paper_2508_11385_amd import tuner
    train = tuner.sample_signatures(160, seed=101, depth_hi=6, dim_hi=4096)
    test = tuner.sample_signatures(60, seed=102, depth_hi=6, dim_hi=4096)
    h_tr, f_tr = tuner.prepare_all(train, workers=8)
    h_te, f_te = tuner.prepare_all(test, workers=8)
    tab_tr = tuner.time_tables(train, h_tr, f_tr, reps=5, seed=1)
    tab_te = tuner.time_tables(test, h_te, f_te, reps=5, seed=2)
    X, y = tuner.dataset(train, h_tr, tab_tr, configs_per_sig=None, seed=3)   # every timed configuration
    init = tuner.he_init(8, n_models=3)
    ones = np.ones(len(y), np.float32)
    cm, losses = cc.coot_costmodel_train(X, y, ones, init, 64, 64, 150, 256, 9, 1e-3, n_models=3)
    cm0, _ = cc.coot_costmodel_train(X, y, ones, init, 64, 64, 0, 256, 9, 1e-3, n_models=3)
    assert losses[-1] < 0.5 * losses[0]
    P, _ = tuner.picks(cm, test, h_te, tab_te)
    Pa, _ = tuner.picks(cm, test, h_te, tab_te, margin=0.0)
    P0, _ = tuner.picks(cm0, test, h_te, tab_te, margin=0.0)
    r_pol = tuner.summarize(tuner.regrets_from_table(tab_te, P[:, 1]))
    r_def = tuner.summarize(tuner.regrets_from_table(tab_te, P[:, 2]))
    r_arg = tuner.summarize(tuner.regrets_from_table(tab_te, Pa[:, 1]))
    r_unt = tuner.summarize(tuner.regrets_from_table(tab_te, P0[:, 1]))
    print(f"in-table regret on {len(test)} held-out signatures ({len(y)} training rows): cost-model policy {r_pol}, "
          f"default {r_def}, trained argmin {r_arg}, untrained argmin {r_unt}", flush=True)
    assert r_pol["geomean"] <= r_def["geomean"] + 0.015, (r_pol, r_def)
    assert r_pol["geomean"] <= 0.12, (r_pol, r_def)
    assert r_arg["geomean"] <= 0.8 * r_unt["geomean"], (r_arg, r_unt)
    for h in h_tr + h_te:
        cc.coot_expr_release(h)
    cc.coot_costmodel_release(cm)
    cc.coot_costmodel_release(cm0)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_dimension_tuning_module_matches_oracle(env, dtype):
    """The tuning module's sum / mean / variance along each dimension (every tile shape,
    vector width and tiles per CU of the tiled space, stage 2 included), launched through
    coot_tune_launch on a ragged shape with a transposed leaf, against the oracle; then
    coot_tune's exhaustive pick, evaluated through coot_reduce, against the oracle too."""
    coot, cc, torch = env
    from oracle import reduce as rd
    R, C = 300, 170
    A, B, Cm, D = synth.matrix_inputs(n_rows=R, n_cols=C, dtype=dtype)
    gs = [coot.Mat.from_numpy(m) for m in (A, B, Cm, D)]
    e = 2.0 * gs[0] + gs[1] % gs[2] - coot.trans(gs[3])
    flat = coot.flatten(e)
    h = coot.frontend.compiled(flat)
    ops = [m.operand() for m in flat.mats]
    Zo = ew.evaluate(flat.postfix, [A, B, Cm, D], flat.scalars, dtype)   # the leaves appear once, in this order
    tol = 1e-6 if dtype == "f32" else 1e-12
    space = cc.coot_tune_space(1)
    for kind, dim in ((cc.COOT_RED_SUM, 0), (cc.COOT_RED_SUM, 1), (cc.COOT_RED_MEAN_DIM, 0), (cc.COOT_RED_VAR_DIM, 1)):
        n_out = C if dim == 0 else R
        out = coot.Mat.empty(1, n_out, dtype, "row") if dim == 0 else coot.Mat.empty(n_out, 1, dtype, "col")
        if kind == cc.COOT_RED_VAR_DIM:
            want = rd.var_dim(Zo, dim, dtype, 0)
            scale = [abs(float(w)) for w in want]
        else:
            want = rd.sum_dim(Zo, dim, dtype) if kind == cc.COOT_RED_SUM else rd.mean_dim(Zo, dim, dtype)
            cnt = R if dim == 0 else C
            scale = [rd.sum_abs(v) / (1 if kind == cc.COOT_RED_SUM else cnt) for v in (Zo.T if dim == 0 else Zo)]
        ok = cc.coot_tune_runnable(h, ops, out.operand(), kind, space, dim=dim)
        assert sum(ok) >= 30
        for cfg, run in zip(space, ok):
            if not run:
                continue
            out.tensor.fill_(float("nan"))
            cc.coot_tune_launch(h, ops, flat.scalars, out.operand(), kind, cfg, dim=dim)
            torch.cuda.synchronize()
            got = out.numpy().ravel()
            for g, w, sc in zip(got, want, scale):
                assert rd.rel_err(float(g), w, sc) <= tol, (kind, dim, cfg)
        best, us = cc.coot_tune(h, ops, flat.scalars, out.operand(), kind, 1, dim=dim)
        assert best in [tuple(c) for c in space] and us > 0
        got = coot.frontend._reduce(e, kind, dim, False, lambda r, c: (1, c) if dim == 0 else (r, 1), best,
                                    False).numpy().ravel()
        for g, w, sc in zip(got, want, scale):
            assert rd.rel_err(float(g), w, sc) <= tol, (kind, dim, best)


def test_library_default_tile_follows_the_output_size(env):
    """Without a configuration the library tiles element-wise evaluation and accu with
    32 x 32 tiles below 2^22 elements and 64 x 64 from there, and reductions along a
    dimension with 64 x 32 (coot_tune's policy 0 reports the default it launches, which
    the tuner's stand-in names too), 32 x 32 where the staging of 64 x 64 tiles does not
    fit; the default launches match the oracle."""
    coot, cc, torch = env
    from paper_2508_11385_amd import tuner
    space = cc.coot_tune_space(1)
    for R, C in ((2048, 2047), (2048, 2048)):
        A, _, _, D = synth.matrix_inputs(n_rows=R, n_cols=C)
        gA, gD = coot.Mat.from_numpy(A), coot.Mat.from_numpy(D)
        e = gA + coot.trans(gD)
        flat = coot.flatten(e)
        h = coot.frontend.compiled(flat)
        ops = [m_.operand() for m_ in flat.mats]
        ts = 64 if R * C >= 1 << 22 else 32
        out = coot.Mat.empty(R, C)
        d, _ = cc.coot_tune(h, ops, flat.scalars, out.operand(), -1, 0)
        assert d[4:] == (ts, ts), (R, C, d)
        assert space[tuner.default_index(space, "f32", None, R * C, -1)] == d
        acc = coot.Mat.empty(1, 1)
        d, _ = cc.coot_tune(h, ops, flat.scalars, acc.operand(), cc.COOT_RED_ACCU, 0)
        assert d[4:] == (ts, ts), (R, C, d)
        s0 = coot.Mat.empty(1, C, "f32", "row")
        d, _ = cc.coot_tune(h, ops, flat.scalars, s0.operand(), cc.COOT_RED_SUM, 0, dim=0)
        assert d[4:] == (64, 32), (R, C, d)
        want = ew.evaluate(flat.postfix, [A, D], flat.scalars, "f32")
        got = coot.eval(e).numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, want), (R, C)
        del gA, gD, out
    # two transposed fp64 leaves stage 2 x 64 x 65 x 8 bytes > 64 KiB on 64 x 64 tiles:
    # the default falls back to 32 x 32 at any size
    A, B, _, D = synth.matrix_inputs(dtype="f64", n_rows=2048, n_cols=2048)
    gA, gB, gD = (coot.Mat.from_numpy(m) for m in (A, B, D))
    e = gA + coot.trans(gB) - coot.trans(gD)
    flat = coot.flatten(e)
    h = coot.frontend.compiled(flat)
    ops = [m_.operand() for m_ in flat.mats]
    d, _ = cc.coot_tune(h, ops, flat.scalars, coot.Mat.empty(2048, 2048, "f64").operand(), -1, 0)
    assert d[4:] == (32, 32), d
    src = {id(gA): A, id(gB): B, id(gD): D}
    want = ew.evaluate(flat.postfix, [src[id(m_)] for m_ in flat.mats], flat.scalars, "f64")
    got = coot.eval(e).numpy()
    torch.cuda.synchronize()
    assert np.array_equal(got, want)
