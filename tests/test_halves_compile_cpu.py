"""CPU guard for the generated 16-bit kernels: random f16 / bf16 expression trees are
generated and compiled by hipRTC for gfx950 (COOT_PF_COMPILE_ONLY: into the caches,
no code object loaded, no device) in every evaluation mode and both families (flat
trees, and trees with transposed leaves that take the tiled kernels).

Compiler combining of the narrowing and widening conversions around the operators
once crashed instruction selection inside hipRTC, which aborts the calling process;
in a GPU test run that takes every test of the process with it.  This test finds such a
crash here, before any device run."""
import pytest

import synth


@pytest.fixture(scope="module")
def cc():
    from paper_2508_11385_amd import _coot
    return _coot


def _modes(cc):
    return [(-1, -1, 0), (cc.COOT_RED_ACCU, -1, 0), (cc.COOT_RED_ACCU, -1, cc.COOT_RF_PLAIN),
            (cc.COOT_RED_SUM, 0, 0), (cc.COOT_RED_SUM, 1, 0), (cc.COOT_RED_NORM, -1, 0),
            (cc.COOT_RED_MAX, -1, 0), (cc.COOT_RED_VAR, -1, 0), (cc.COOT_RED_MEAN_DIM, 1, 0),
            (cc.COOT_RED_VAR_DIM, 0, 0)]


# (seed, depth, operands, square): square shapes let the generator place transposed leaves
TREES = [(s, d, k, sq) for s, (d, k, sq) in enumerate([(2, 2, True), (3, 3, False), (4, 4, True), (5, 5, True),
                                                         (6, 3, False)])]


@pytest.mark.parametrize("dt", ["f16", "bf16"])
@pytest.mark.parametrize("tree", range(len(TREES)))
def test_random_16bit_trees_compile_in_every_mode(cc, dt, tree, tmp_path, monkeypatch):
    monkeypatch.setenv("COOT_CACHE_DIR", str(tmp_path))
    seed, depth, k, square = TREES[tree]
    g = synth.rng_for(31, seed, 1 if dt == "bf16" else 0)
    spec = synth.random_tree(g, depth, k, 24, 24 if square else 40, dt)
    slots = [(cc.DTYPE_CODE[dt], 0)] * len(spec.slot_shapes)
    h = cc.coot_expr_compile(spec.postfix, slots, len(spec.scalars))
    modes = _modes(cc)
    try:
        # every tree compiles element-wise with its narrowest and widest groups; the
        # reductions rotate over the trees, so that each dtype covers every mode twice
        for v in (1, 8):
            cc.coot_expr_prepare(h, -1, -1, cc.COOT_PF_COMPILE_ONLY, (v, 0, 0, 0))
        for j in range(4):
            mode, dim, rf = modes[1 + (4 * tree + j) % (len(modes) - 1)]
            cc.coot_expr_prepare(h, mode, dim, rf | cc.COOT_PF_COMPILE_ONLY)
    finally:
        cc.coot_expr_release(h)
