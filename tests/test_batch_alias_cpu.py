"""Overlap rules of a batch, checked on the host before any device work (so these
run without a GPU on fake addresses): every expression of a batch runs at the same
time as every other, so an output may overlap nothing but an operand of its own
expression read untransposed with the output's own layout (in place)."""
import pytest


@pytest.fixture(scope="module")
def cc():
    from paper_2508_11385_amd import _coot
    return _coot


ADD = [("load", 0), ("load", 1), ("add",)]
TADD = [("load", 0), ("trans",), ("load", 1), ("add",)]
MB = 1 << 20


def _m(cc, addr, r, c, ld=None):
    return cc.coot_operand(addr, r, c, ld or r, cc.COOT_F32, cc.COOT_MAT)


def _create(cc, exprs, ops, outs):
    return cc.coot_batch_create(exprs, ops, [[] for _ in exprs], outs)


def _status(cc, fn):
    try:
        fn()
    except cc.CootError as e:
        return e.status, str(e)
    return cc.COOT_OK, ""


def test_overlapping_batches_are_refused(cc):
    h = cc.coot_expr_compile(ADD, [(cc.COOT_F32, 0)] * 2, 0)
    ht = cc.coot_expr_compile(TADD, [(cc.COOT_F32, 0)] * 2, 0)
    A, B, O1, O2 = 16 * MB, 32 * MB, 48 * MB, 64 * MB        # 64 x 64 fp32 = 16 KiB each, far apart
    cases = {
        # two outputs sharing a byte
        "outputs overlap": ([h, h], [[_m(cc, A, 64, 64), _m(cc, B, 64, 64)]] * 2,
                            [_m(cc, O1, 64, 64), _m(cc, O1 + 64 * 64 * 4 - 4, 64, 64)]),
        # expression 1 reads what expression 0 writes
        "reads another's output": ([h, h], [[_m(cc, A, 64, 64), _m(cc, B, 64, 64)],
                                            [_m(cc, O1, 64, 64), _m(cc, B, 64, 64)]],
                                   [_m(cc, O1, 64, 64), _m(cc, O2, 64, 64)]),
        # a submatrix view of an operand as the output (shifted by one column)
        "shifted view of an operand": ([h], [[_m(cc, A, 64, 64, 128), _m(cc, B, 64, 64)]],
                                       [_m(cc, A + 64 * 4, 64, 64, 128)]),
        # in place, but the operand is read transposed
        "in place on a transposed leaf": ([ht], [[_m(cc, A, 64, 64), _m(cc, B, 64, 64)]], [_m(cc, A, 64, 64)]),
    }
    for name, (ex, ops, outs) in cases.items():
        st, msg = _status(cc, lambda: _create(cc, ex, ops, outs))
        assert st == cc.COOT_EALIAS, (name, st, msg)


def test_disjoint_and_in_place_batches_pass_the_overlap_check(cc):
    """Without a device, a batch that passes the checks fails later, at its first HIP
    call (COOT_EHIP), not with COOT_EALIAS."""
    h = cc.coot_expr_compile(ADD, [(cc.COOT_F32, 0)] * 2, 0)
    A, B, O1, O2 = 16 * MB, 32 * MB, 48 * MB, 64 * MB
    ok_cases = [
        # shared read-only operands, disjoint outputs; adjacent (touching) outputs
        ([h, h], [[_m(cc, A, 64, 64), _m(cc, B, 64, 64)]] * 2,
         [_m(cc, O1, 64, 64), _m(cc, O1 + 64 * 64 * 4, 64, 64)]),
        # in place: y = a + y with the output's own layout
        ([h, h], [[_m(cc, A, 64, 64), _m(cc, O1, 64, 64)], [_m(cc, B, 64, 64), _m(cc, O2, 64, 64)]],
         [_m(cc, O1, 64, 64), _m(cc, O2, 64, 64)]),
    ]
    for ex, ops, outs in ok_cases:
        st, msg = _status(cc, lambda: _create(cc, ex, ops, outs))
        assert st != cc.COOT_EALIAS, msg
