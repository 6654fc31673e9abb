"""CPU checks of the tiled kernels' launch planning: the vector width the library
plans for a tile fits it (the tile's 256 threads cover whole column segments in at
most as many passes as the tile has columns), and a kernel instance whose vector
width does not fit its tile is refused at compile time.  No device is needed."""
import re

import pytest


@pytest.fixture(scope="module")
def cc():
    from paper_2508_11385_amd import _coot
    return _coot


def _expr(cc, dt, n_p1):
    """sum of n_p1 transposed leaves and one untransposed leaf (n_p1 + 1 slots)."""
    post = [("load", 0)]
    for k in range(n_p1):
        post += [("load", k + 1), ("trans",), ("add",)]
    slots = [(cc.DTYPE_CODE[dt], 0)] * (n_p1 + 1)
    return cc.coot_expr_compile(post, slots, 0)


def _vt(name):
    """(vector width, tile rows, tile columns) of a tiled kernel's name"""
    m = re.search(r"_v(\d+)t(\d+)x(\d+)", name)
    assert m, name
    return int(m.group(1)), int(m.group(2)), int(m.group(3))


@pytest.mark.parametrize("dt", ["f16", "bf16", "f32", "f64"])
@pytest.mark.parametrize("n_p1", [1, 4])
def test_planned_vector_width_fits_the_tile(cc, dt, n_p1):
    h = _expr(cc, dt, n_p1)
    vecs = (1, 2, 4, 8) if dt in ("f16", "bf16") else (1, 2, 4)
    modes = [(-1, -1), (cc.COOT_RED_ACCU, -1), (cc.COOT_RED_SUM, 0), (cc.COOT_RED_SUM, 1),
             (cc.COOT_RED_MEAN_DIM, 0), (cc.COOT_RED_VAR_DIM, 1)]
    if dt in ("u32", "s32"):
        modes = modes[:4]
    for mode, dim in modes:
        for v in vecs:
            V, TR, TC = _vt(cc.coot_expr_kernel_name(h, mode, dim, (v, 0, 0, 0)))
            assert V <= v and V * 256 <= TR * TC, (mode, dim, v, V, TR, TC)
            for tile in ((128, 32), (32, 128), (256, 16), (16, 256)):
                try:
                    V, TR, TC = _vt(cc.coot_expr_kernel_name(h, mode, dim, (v, 0, 0, 0) + tile))
                except cc.CootError as e:     # a tile whose staged leaves exceed the LDS budget
                    assert e.status == cc.COOT_EINVAL
                    assert n_p1 == 4
                    continue
                assert (TR, TC) == tile and V <= v and V * 256 <= TR * TC, (mode, dim, v, V, TR, TC)
    cc.coot_expr_release(h)


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_four_transposed_16bit_leaves_compile_with_their_widest_groups(cc, dt, tmp_path, monkeypatch):
    """Four transposed 16-bit leaves (staged in binary32) cannot stage on the default
    64 x 64 tile of the 16-bit types and take 32 x 32, where 16-byte groups (8 elements)
    would leave a pass wider than the tile: the library plans 4-element groups, for
    element-wise evaluation, full reductions and reductions along a dimension, and every
    one compiles."""
    monkeypatch.setenv("COOT_CACHE_DIR", str(tmp_path))
    h = _expr(cc, dt, 4)
    for mode, dim in ((-1, -1), (cc.COOT_RED_ACCU, -1), (cc.COOT_RED_SUM, 0), (cc.COOT_RED_SUM, 1),
                      (cc.COOT_RED_VAR_DIM, 0)):
        assert _vt(cc.coot_expr_kernel_name(h, mode, dim, (8, 0, 0, 0))) == (4, 32, 32), (mode, dim)
        cc.coot_expr_prepare(h, mode, dim, cc.COOT_PF_COMPILE_ONLY, (8, 0, 0, 0))
    cc.coot_expr_release(h)


def test_a_vector_width_wider_than_the_tile_is_refused(cc):
    """The tile walks assert at compile time that their passes cover the tile."""
    h = _expr(cc, "f16", 4)
    with pytest.raises(cc.CootError) as e:
        cc.coot_debug_codegen(h, cc.COOT_RED_SUM, 0, 0, 1, 8, 0, 32, True)
    assert e.value.status == cc.COOT_ECOMPILE
    assert "passes must cover" in str(e.value)
    src, size = cc.coot_debug_codegen(h, cc.COOT_RED_SUM, 0, 0, 1, 4, 0, 32, True)
    assert size > 1000
    cc.coot_expr_release(h)


def test_tile_arguments_are_checked(cc):
    h = _expr(cc, "f32", 1)
    for bad in ((4, 0, 0, 0, 64, 0), (4, 0, 0, 0, 48, 64), (4, 0, 0, 0, 16, 32), (4, 0, 0, 0, 512, 16),
                (4, 0, 0, 0, 256, 64)):
        with pytest.raises(cc.CootError) as e:
            cc.coot_expr_kernel_name(h, -1, -1, bad)
        assert e.value.status == cc.COOT_EINVAL, bad
    # five transposed fp64 leaves do not fit 64 x 64 staging (5 x 64 x 65 x 8 bytes)
    h5 = _expr(cc, "f64", 5)
    assert _vt(cc.coot_expr_kernel_name(h5, -1, -1, None))[1:] == (32, 32)
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_kernel_name(h5, -1, -1, (2, 0, 0, 0, 64, 64))
    assert e.value.status == cc.COOT_EINVAL
    cc.coot_expr_release(h)
    cc.coot_expr_release(h5)


@pytest.mark.parametrize("dt", ["u32", "s32", "f32", "f64"])
def test_tuner_default_index_names_the_library_default(cc, dt):
    """The tuner's stand-in for "no tuner" is an entry of each family's configuration
    space (six fields: vec, ept, waves, workgroups per CU, tile rows, tile columns), with
    the library's fallbacks where the operands rule the default out (NaN times)."""
    import numpy as np
    from paper_2508_11385_amd import tuner
    v = 2 if dt == "f64" else 4
    flat, tiled = cc.coot_tune_space(0), cc.coot_tune_space(1)
    assert all(len(c) == 6 for c in flat + tiled)
    assert flat[tuner.default_index(flat, dt, None, 1000, -1)] == (v, 1, 4, 4, 0, 0)
    assert flat[tuner.default_index(flat, dt, None, 1 << 25, -1)] == (2, 8, 4, 16, 0, 0)
    big_red = (2, 4, 8, 8, 0, 0) if dt == "f64" else (4, 4, 4, 2, 0, 0)
    assert flat[tuner.default_index(flat, dt, None, 1 << 25, 0)] == big_red
    assert tiled[tuner.default_index(tiled, dt, None, 1000, -1)] == (2, 1, 4, 8, 32, 32)
    t = np.ones(len(tiled))
    t[tiled.index((2, 1, 4, 8, 32, 32))] = np.nan   # operands that rule out 2-element groups
    assert tiled[tuner.default_index(tiled, dt, t, 1000, -1)] == (1, 1, 4, 8, 32, 32)
    # from 2^22 elements the tiled default is 64 x 64; its fallbacks: scalar accesses, then
    # 32 x 32 tiles where the staging of 64 x 64 ones does not fit
    big = 1 << 22
    assert tiled[tuner.default_index(tiled, dt, None, big - 1, -1)] == (2, 1, 4, 8, 32, 32)
    assert tiled[tuner.default_index(tiled, dt, None, big, -1)] == (2, 1, 4, 8, 64, 64)
    assert tiled[tuner.default_index(tiled, dt, None, big, 0)] == (2, 1, 4, 8, 64, 64)
    t = np.ones(len(tiled))
    t[tiled.index((2, 1, 4, 8, 64, 64))] = np.nan
    assert tiled[tuner.default_index(tiled, dt, t, big, -1)] == (1, 1, 4, 8, 64, 64)
    t[tiled.index((1, 1, 4, 8, 64, 64))] = np.nan
    assert tiled[tuner.default_index(tiled, dt, t, big, -1)] == (2, 1, 4, 8, 32, 32)
    t[tiled.index((2, 1, 4, 8, 32, 32))] = np.nan
    assert tiled[tuner.default_index(tiled, dt, t, big, -1)] == (1, 1, 4, 8, 32, 32)
    t = np.ones(len(flat))
    t[flat.index((v, 1, 4, 4, 0, 0))] = np.nan   # misaligned operands: scalar accesses
    assert flat[tuner.default_index(flat, dt, t, 1000, -1)] == (1, 1, 4, 4, 0, 0)


def test_timing_tables_are_saved_with_whole_configurations(cc, tmp_path):
    """The tuner's table dump keeps all six fields of each configuration next to its
    time and features (plain arrays, loadable without pickling)."""
    import numpy as np
    from paper_2508_11385_amd import tuner
    sigs = tuner.sample_signatures(3, seed=77)
    handles = [tuner._handle(spec) for spec, _ in sigs]
    space = cc.coot_tune_space(1)[:5]
    tables = [(space, [10.0 + i + 0.5 * k for k in range(len(space))]) for i in range(len(sigs))]
    path = str(tmp_path / "t.npz")
    tuner.save_tables(path, sigs, [1] * len(sigs), handles, tables, [0, 0, 1])
    z = np.load(path)
    assert z["cfg"].shape == (3 * len(space), 6)
    assert [tuple(r) for r in z["cfg"][:len(space)]] == [tuple(c) for c in space]
    assert np.allclose(z["us"], np.concatenate([t for _, t in tables]))
    assert z["feat"].shape[0] == 3 * len(space) and z["meta"].shape == (3, 9)
    for h in handles:
        cc.coot_expr_release(h)


def test_library_default_tiles(cc):
    """Without a configuration the tiled kernels take, for outputs below 2^22 elements
    (the names are planned for 1 x 1 operands), 32 x 32 tiles for element-wise evaluation
    and full reductions, 64 x 32 for reductions along a dimension, 64 x 64 for 16-bit
    types; 32 x 32 where the staged transposed leaves would not fit; and a request whose
    staging does not fit even 32 x 32 (eight transposed fp64 leaves) is refused."""
    for dt, n_p1, want_eval, want_dim in (("f32", 1, (32, 32), (64, 32)), ("f64", 1, (32, 32), (64, 32)),
                                          ("u32", 1, (32, 32), (64, 32)), ("f64", 4, (32, 32), (32, 32)),
                                          ("f16", 1, (64, 64), (64, 64)), ("bf16", 4, (32, 32), (32, 32))):
        h = _expr(cc, dt, n_p1)
        assert _vt(cc.coot_expr_kernel_name(h, -1, -1))[1:] == want_eval, (dt, n_p1)
        assert _vt(cc.coot_expr_kernel_name(h, cc.COOT_RED_ACCU, -1))[1:] == want_eval, (dt, n_p1)
        for dim in (0, 1):
            assert _vt(cc.coot_expr_kernel_name(h, cc.COOT_RED_SUM, dim))[1:] == want_dim, (dt, n_p1, dim)
        cc.coot_expr_release(h)
    h = _expr(cc, "f64", 7)                     # 7 x 32 x 33 x 8 B = 59136 B: fits
    assert _vt(cc.coot_expr_kernel_name(h, -1, -1))[1:] == (32, 32)
    cc.coot_expr_release(h)
    h = _expr(cc, "f64", 8)                     # 8 x 32 x 33 x 8 B = 67584 B > 64 KiB
    with pytest.raises(cc.CootError) as e:
        cc.coot_expr_kernel_name(h, -1, -1)
    assert e.value.status == cc.COOT_EUNSUPPORTED and "64 KiB" in str(e.value)
    cc.coot_expr_release(h)
