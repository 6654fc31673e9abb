"""CPU-only checks of the C ABI: the library loads, exports every symbol the
header declares, validates expressions and shapes, and every generated kernel
family compiles for gfx950 through hipRTC (no device needed)."""
import ctypes

import numpy as np
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cc():
    from paper_2508_11385_amd import _coot
    return _coot


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "coot.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(coot_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(cc):
    syms = _declared_symbols()
    assert "coot_expr_eval" in syms and "coot_reduce" in syms
    lib = ctypes.CDLL(cc.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s
    for s in syms:
        assert s in cc.EXPORTED, f"binding lacks {s}"


def _ops(n, dt="f32", kind=0):
    return [(cc_mod().DTYPE_CODE[dt], kind)] * n


def cc_mod():
    from paper_2508_11385_amd import _coot
    return _coot


Z = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",), ("load", 3),
     ("trans",), ("sub",)]
W = [("load", 0), ("exp",), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]


def test_validation_errors(cc):
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_compile([("load", 0), ("add",)], _ops(1), 0)
    assert e.value.status == cc.COOT_EINVAL
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_compile([("load", 0), ("exp",)], _ops(1, "u32"), 0)
    assert e.value.status == cc.COOT_ETYPE
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_compile([("load", 0), ("load", 1), ("add",)], [(cc.COOT_F32, 0), (cc.COOT_F64, 0)], 0)
    assert e.value.status == cc.COOT_ETYPE
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_compile([("load", 3)], _ops(1), 0)
    assert e.value.status == cc.COOT_EINVAL
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_compile([("scalar", 0)], [], 0)
    assert e.value.status == cc.COOT_EINVAL
    h = cc.coot_expr_compile(Z, _ops(4), 1)
    cc.coot_expr_release(h)


def _opnd(cc, r, c, dt="f32", kind=0):
    return cc.coot_operand(0x1000, r, c, r, cc.DTYPE_CODE[dt], kind)


def test_shape_inference(cc):
    h = cc.coot_expr_compile(Z, _ops(4), 1)
    assert cc.coot_expr_out_shape(h, [_opnd(cc, 7, 5)] * 3 + [_opnd(cc, 5, 7)]) == (7, 5)
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_out_shape(h, [_opnd(cc, 7, 5)] * 4)
    assert e.value.status == cc.COOT_ESHAPE
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_out_shape(h, [_opnd(cc, 7, 5, "f64")] * 3 + [_opnd(cc, 5, 7, "f64")])
    assert e.value.status == cc.COOT_ETYPE
    # a Col must have one column
    hc = cc.coot_expr_compile([("load", 0)], [(cc.COOT_F32, cc.COOT_COL)], 0)
    with pytest.raises(cc.CootError):
        cc.coot_expr_out_shape(hc, [cc.coot_operand(0x1000, 4, 2, 4, cc.COOT_F32, cc.COOT_COL)])
    # trans(trans(A)) keeps the shape, trans(A) swaps it
    ht = cc.coot_expr_compile([("load", 0), ("trans",)], _ops(1), 0)
    assert cc.coot_expr_out_shape(ht, [_opnd(cc, 3, 8)]) == (8, 3)


FAMILIES = [
    # (postfix, n_slots, n_scalars, mode, dim, fam, vec, ept, tile edge or (rows, cols), dtype)
    (Z, 4, 1, -1, -1, 1, 4, 0, 64, "f32"),
    (Z, 4, 1, -1, -1, 1, 2, 0, 32, "f64"),
    (W, 2, 1, -1, -1, 0, 4, 4, 0, "f32"),
    (W, 2, 1, -1, -1, 0, 2, 2, 0, "f64"),
    ([("load", 0), ("load", 1), ("schur",)], 2, 0, 2, -1, 0, 4, 4, 0, "f32"),
    ([("load", 0)], 1, 0, 3, -1, 0, 4, 8, 0, "f32"),
    ([("load", 0)], 1, 0, 0, -1, 0, 4, 4, 0, "u32"),
    (Z, 4, 1, 1, 0, 1, 4, 0, 64, "f32"),
    (Z, 4, 1, 1, 1, 1, 4, 0, 64, "f32"),
    (Z, 4, 1, 0, -1, 1, 4, 0, 64, "f64"),
    ([("load", 0), ("load", 1), ("add",), ("load", 2), ("schur",)], 3, 0, -1, -1, 0, 4, 4, 0, "u32"),
    ([("load", 0), ("scalar", 0), ("load", 1), ("schur",), ("sub",)], 2, 1, -1, -1, 0, 4, 4, 0, "s32"),
    (Z, 4, 1, -1, -1, 1, 4, 0, 64, "f16"),
    (W, 2, 1, -1, -1, 0, 4, 4, 0, "bf16"),
    (Z, 4, 1, 1, 0, 1, 4, 0, 64, "bf16"),
    (Z, 4, 1, 0, -1, 1, 4, 0, 64, "f16"),
    ([("load", 0)], 1, 0, 3, -1, 0, 4, 8, 0, "f16"),
    ([("load", 0), ("load", 1), ("schur",)], 2, 0, 2, -1, 0, 4, 4, 0, "bf16"),
    (Z, 4, 1, 4, -1, 1, 4, 0, 64, "f32"),     # min, tiled
    (W, 2, 1, 5, -1, 0, 4, 4, 0, "f64"),      # max, flat
    ([("load", 0)], 1, 0, 5, -1, 0, 4, 4, 0, "s32"),
    (W, 2, 1, 6, -1, 0, 4, 4, 0, "f32"),      # mean
    (Z, 4, 1, 7, -1, 1, 2, 0, 32, "f64"),     # norm1
    (W, 2, 1, 8, -1, 0, 8, 1, 0, "f16"),      # norm_inf
    (Z, 4, 1, 9, 0, 1, 4, 0, 64, "f32"),      # mean along dim 0
    (Z, 4, 1, 9, 1, 1, 8, 0, 64, "bf16"),     # mean along dim 1
    (W, 2, 1, 10, -1, 0, 4, 4, 0, "f32"),     # var, flat (two passes)
    (Z, 4, 1, 10, -1, 1, 2, 0, 64, "f64"),    # var, tiled
    (W, 2, 1, 10, -1, 0, 8, 1, 0, "f16"),     # var, 16-bit
    (Z, 4, 1, 11, 0, 1, 4, 0, 64, "f32"),     # var along dim 0
    (Z, 4, 1, 11, 1, 1, 2, 0, 32, "f64"),     # var along dim 1
    # rectangular tiles (rows x columns)
    (Z, 4, 1, -1, -1, 1, 4, 0, (128, 32), "f32"),
    (Z, 4, 1, -1, -1, 1, 2, 0, (32, 128), "f64"),
    (Z, 4, 1, 1, 0, 1, 4, 0, (256, 16), "f32"),
    (Z, 4, 1, 1, 1, 1, 4, 0, (128, 64), "f32"),
    (Z, 4, 1, 11, 0, 1, 8, 0, (128, 32), "bf16"),
    (Z, 4, 1, 0, -1, 1, 4, 0, (32, 128), "f16"),
    (Z, 4, 1, 3, -1, 1, 1, 0, (16, 256), "f32"),   # norm (with its rescaled pass)
]


@pytest.mark.parametrize("case", range(len(FAMILIES)))
def test_codegen_compiles_for_gfx950(cc, case):
    post, ns, nsc, mode, dim, fam, vec, ept, ts, dt = FAMILIES[case]
    h = cc.coot_expr_compile(post, _ops(ns, dt), nsc)
    src, size = cc.coot_debug_codegen(h, mode, dim, 0, fam, vec, ept, ts, True)
    assert size > 1000
    assert 'extern "C" __global__' in src
    if mode < 0 and any(p[0] == "trans" for p in post):
        assert "tiled_eval" in src
    cc.coot_expr_release(h)


def test_half_types_round_each_operator_and_stay_out_of_the_cost_model(cc):
    for dt in ("f16", "bf16"):
        h = cc.coot_expr_compile(W, _ops(2, dt), 1)
        src, _ = cc.coot_debug_codegen(h, -1, -1, 0, 0, 4, 1, 0, False)
        assert f"typedef coot::{dt} S;" in src
        start = src.index("T f(const T* L")
        body = src[start:src.index("return t", start)]
        assert body.count("coot::St<S>::rnd(") == 4          # exp, abs, +, /: each rounded to the type
        with pytest.raises(cc.CootError) as e:
            cc.coot_costmodel_features(h, 8, 8, 0, [(4, 1, 4, 4)])
        assert e.value.status == cc.COOT_EUNSUPPORTED
        cc.coot_expr_release(h)


def test_generated_body_has_one_statement_per_operator(cc):
    h = cc.coot_expr_compile(Z, _ops(4), 1)
    src, _ = cc.coot_debug_codegen(h, -1, -1, 0, 1, 4, 0, 64, False)
    start = src.index("T f(const T* L")
    body = src[start:src.index("return t", start)]
    # 4 leaf reads + 1 scalar + 4 arithmetic operators; trans costs nothing
    assert body.count("const T t") == 9
    assert body.count("op_") == 4
    assert "NP1 = 1" in src
    cc.coot_expr_release(h)


def test_random_trees_generate_and_leaf_parities(cc):
    g = synth.rng_for(77)
    for _ in range(40):
        spec = synth.random_tree(g, int(g.integers(1, 8)), int(g.integers(2, 6)), 9, 13, "f32")
        slots = [(cc.COOT_F32, 0)] * len(spec.slot_shapes)
        h = cc.coot_expr_compile(spec.postfix, slots, len(spec.scalars))
        ops = [_opnd(cc, r, c) for r, c in spec.slot_shapes]
        assert cc.coot_expr_out_shape(h, ops) == (9, 13)
        src, _ = cc.coot_debug_codegen(h, -1, -1, 0, 1, 1, 0, 64, False)
        n_p1 = int(re.search(r"NP1 = (\d+)", src).group(1))
        transposed_slots = {k for k, (r, c) in enumerate(spec.slot_shapes) if (r, c) == (13, 9)}
        assert n_p1 == len(transposed_slots)
        cc.coot_expr_release(h)


def test_costmodel_features_match_oracle_definition(cc):
    from oracle import features as of
    g = synth.rng_for(78)
    space = cc.coot_tune_space(0) + cc.coot_tune_space(1)
    assert len(cc.coot_tune_space(0)) == 192 and len(cc.coot_tune_space(1)) == 144
    for trial in range(25):
        dt = ["u32", "s32", "f32", "f64"][trial % 4]
        r, c = int(g.integers(1, 20000)), int(g.integers(1, 20000))
        spec = synth.random_tree(g, int(g.integers(1, 9)), int(g.integers(2, 6)), 7, 7, dt)
        h = cc.coot_expr_compile(spec.postfix, [(cc.DTYPE_CODE[dt], 0)] * len(spec.slot_shapes), len(spec.scalars))
        red = trial % 4
        cfgs = [space[k] for k in g.integers(0, len(space), 7)]
        got = cc.coot_costmodel_features(h, r, c, red, cfgs)
        for k, cfg in enumerate(cfgs):
            want = of.features(spec.postfix, dt, r, c, of.RED_ORDER[red], cfg)
            assert np.allclose(got[k], want, rtol=1e-6, atol=1e-6), (spec.postfix, got[k], want)
        cc.coot_expr_release(h)


def test_tuning_module_compiles_every_variant(cc):
    h = cc.coot_expr_compile(W, _ops(2), 1)
    assert cc.coot_tune_prepare(h, [_opnd(cc, 100, 50)] * 2, -1) == 0
    hz = cc.coot_expr_compile(Z, _ops(4), 1)
    assert cc.coot_tune_prepare(hz, [_opnd(cc, 100, 50)] * 3 + [_opnd(cc, 50, 100)], -1) == 1
    hd = cc.coot_expr_compile([("load", 0), ("load", 1), ("schur",)], _ops(2), 0)
    assert cc.coot_tune_prepare(hd, [_opnd(cc, 1000, 1)] * 2, 0) == 0
    with pytest.raises(cc.CootError) as e:
        cc.coot_tune_prepare(hd, [_opnd(cc, 1000, 1)] * 2, 1)
    assert e.value.status == cc.COOT_EUNSUPPORTED
    for dt in ("f16", "bf16"):       # the 16-bit types' tuning modules (every variant) compile too
        hw = cc.coot_expr_compile(W, _ops(2, dt), 1)
        assert cc.coot_tune_prepare(hw, [_opnd(cc, 100, 50, dt)] * 2, -1) == 0
        hz = cc.coot_expr_compile(Z, _ops(4, dt), 1)
        assert cc.coot_tune_prepare(hz, [_opnd(cc, 100, 50, dt)] * 3 + [_opnd(cc, 50, 100, dt)], -1) == 1


def test_runnable_configurations(cc):
    """Vector widths that the operands' alignment or shape forbid are reported, without a device."""
    flat = cc.coot_tune_space(0)
    h = cc.coot_expr_compile(W, _ops(2), 1)
    ok = cc.coot_tune_runnable(h, [_opnd(cc, 100, 50)] * 2, _opnd(cc, 100, 50), -1, flat)
    assert all(ok)
    mis = cc.coot_operand(0x100004, 100, 50, 100, cc.COOT_F32, cc.COOT_MAT)   # 4-byte aligned only
    ok = cc.coot_tune_runnable(h, [mis, _opnd(cc, 100, 50)], _opnd(cc, 100, 50), -1, flat)
    assert all(o == (c[0] == 1) for o, c in zip(ok, flat))
    tiled = cc.coot_tune_space(1)
    assert {(c[4], c[5]) for c in tiled} == {(64, 64), (128, 32), (32, 128), (256, 16), (128, 64), (32, 32),
                                            (64, 16), (16, 64), (128, 8), (256, 8), (128, 16), (64, 32)}
    hz = cc.coot_expr_compile(Z, _ops(4), 1)
    ops = [_opnd(cc, 6, 8)] * 3 + [_opnd(cc, 8, 6)]                            # 6 rows: 2 | 6, 4 does not
    ok = cc.coot_tune_runnable(hz, ops, _opnd(cc, 6, 8), -1, tiled)
    assert all(o == (c[0] in (1, 2)) for o, c in zip(ok, tiled))
    # four transposed fp64 leaves: 128 x 64 tiles would stage 4 x 128 x 65 x 8 bytes > 64 KiB
    h4 = cc.coot_expr_compile([("load", 0), ("trans",), ("load", 1), ("trans",), ("add",), ("load", 2), ("trans",),
                               ("add",), ("load", 3), ("trans",), ("add",)], _ops(4, "f64"), 0)
    ok = cc.coot_tune_runnable(h4, [_opnd(cc, 64, 64, "f64")] * 4, _opnd(cc, 64, 64, "f64"), -1, tiled)
    assert all(o == (c[4] * (c[5] + 1) * 8 * 4 <= 65536) for o, c in zip(ok, tiled))
    with pytest.raises(cc.CootError) as e:
        cc.coot_tune_runnable(hz, ops, None, -1, tiled)
    assert e.value.status == cc.COOT_EINVAL


def test_compile_only_prepare_needs_no_device(cc, tmp_path, monkeypatch):
    """COOT_PF_COMPILE_ONLY generates and compiles into the caches without loading a code
    object, so it runs here without a GPU; the on-disk cache receives the module."""
    import os
    monkeypatch.setenv("COOT_CACHE_DIR", str(tmp_path))
    h = cc.coot_expr_compile([("load", 0), ("scalar", 0), ("schur",), ("load", 1), ("add",)], _ops(2), 1)
    cc.coot_expr_prepare(h, -1, rflags=cc.COOT_PF_COMPILE_ONLY)
    assert any(f.endswith(".co") for f in os.listdir(tmp_path))
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_prepare(h, -1, rflags=0x8000)
    assert e.value.status == cc.COOT_EINVAL
    cc.coot_expr_release(h)


def test_set_allocator_needs_both_functions(cc):
    import ctypes
    f = cc.ALLOC_FN(lambda n, s, ctx: 0)
    with pytest.raises(cc.CootError) as e:
        _ = cc.lib.coot_set_allocator(ctypes.cast(f, ctypes.c_void_p), None, None)
        cc._check(_)
    assert e.value.status == cc.COOT_EINVAL
    with pytest.raises(ValueError):
        cc.coot_set_allocator(lambda n, s: 0, None)


def test_binding_constants_match_the_header():
    """Every COOT_* enumerator and flag of include/coot.h has the same value in the
    Python binding (the binding marshals numbers, so a drift would be silent)."""
    import re
    from paper_2508_11385_amd import _coot as cc
    text = open(os.path.join(ROOT, "include", "coot.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    found = {}
    for name, val in re.findall(r"\b(COOT_[A-Z0-9_]+)\s*=\s*(-?\d+)", text):
        found[name] = int(val)
    for name, val in re.findall(r"#define\s+(COOT_[A-Z0-9_]+)\s+(0x[0-9a-fA-F]+|\d+)u?", text):
        found[name] = int(val, 0)
    checked = 0
    for name, val in found.items():
        if hasattr(cc, name):
            assert getattr(cc, name) == val, name
            checked += 1
    for name in ("COOT_RED_MEAN_DIM", "COOT_RED_VAR", "COOT_RED_VAR_DIM", "COOT_RF_VAR_N", "COOT_RF_PLAIN"):
        assert name in found and hasattr(cc, name), name
    assert checked >= 15
    # op codes: the binding's name -> code table
    ops = {n[len("COOT_OP_"):].lower(): v for n, v in found.items() if n.startswith("COOT_OP_")}
    assert ops and ops == {k: v for k, v in cc.OPCODES.items() if k in ops} and set(ops) <= set(cc.OPCODES)
