"""Exhaustive binary32 check of the kernels' exp (every one of the 2^32 bit patterns),
on the CPU: the device code built for the host against the oracle, chunk by chunk.

The oracle's results over all 2^32 patterns are stored as one SHA-256 digest per
chunk of 2^26 patterns (tests/golden/unary_f32_digests.json, written by
tests/golden/make_unary_digests.py, which calls only the oracle; any NaN result is
hashed as 0x7FC00000).  A digest that differs is resolved by evaluating the oracle
on that chunk and naming the first differing inputs.  The GPU test of the same
digests (exp, sqrt, abs, neg through the fused kernel) is test_gpu_exhaustive.py."""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import elementwise as ew
from tests import hostexp
from tests.golden import make_unary_digests as mud

GOLD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "unary_f32_digests.json")))


def first_differences(op, k, y):
    """Inputs of chunk k where y differs from the oracle (NaN matches NaN)."""
    x = mud.patterns(k)
    with np.errstate(all="ignore"):
        want = ew.evaluate([("load", 0), (op,)], [x.reshape(-1, 1)], [], "f32").ravel()
    bad = ~((y.view(np.uint32) == want.view(np.uint32)) | (np.isnan(y) & np.isnan(want)))
    i = np.flatnonzero(bad)[:5]
    return [(hex(int(x.view(np.uint32)[j])), float(y[j]), float(want[j])) for j in i]


@pytest.mark.parametrize("op,k", [("exp", 33), ("sqrt", 16), ("abs", 40), ("neg", 7)])
def test_stored_digests_are_the_oracles(op, k):
    assert mud.oracle_chunk((op, k)) == GOLD["digests"][op][k]


def test_digest_shape():
    assert GOLD["chunk_bits"] == mud.CHUNK_BITS == 26
    for op in mud.OPS:
        assert len(GOLD["digests"][op]) == mud.N_CHUNKS == 64


@pytest.mark.slow
def test_host_build_of_kernel_exp_on_all_binary32_patterns():
    L = hostexp.build()
    if L is None:
        pytest.skip("g++ not available")

    def run(k):
        x = mud.patterns(k)
        y = np.empty_like(x)
        L.expf_rn_n(x.ctypes.data, y.ctypes.data, x.size)     # ctypes releases the GIL
        return k, y if mud.digest(y) != GOLD["digests"]["exp"][k] else None

    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as pool:
        for k, y in pool.map(run, range(mud.N_CHUNKS)):
            assert y is None, f"chunk {k}: {first_differences('exp', k, y)}"


@pytest.mark.slow
def test_host_build_of_kernel_log_on_all_positive_binary32_patterns():
    """The kernels' binary32 log (float-float arithmetic, no binary64) on every positive
    pattern (2^31 inputs: subnormals, normals, +inf, NaNs) against the oracle's
    correctly rounded log: never more than 1 ulp away, and correctly rounded on all
    but a few dozen inputs (58 when this test was written)."""
    L = hostexp.build()
    if L is None:
        pytest.skip("g++ not available")

    def run(k):
        x = mud.patterns(k)
        y = np.empty_like(x)
        L.logf_n(x.ctypes.data, y.ctypes.data, x.size)
        with np.errstate(all="ignore"):
            want = ew.log_rounded(x, "f32")
        fin = np.isfinite(want)
        spec_ok = bool(np.all((y[~fin] == want[~fin]) | (np.isnan(y[~fin]) & np.isnan(want[~fin]))))
        a = y[fin].view(np.int32).astype(np.int64)
        b = want[fin].view(np.int32).astype(np.int64)
        a = np.where(a < 0, -(a & 0x7FFFFFFF), a)
        b = np.where(b < 0, -(b & 0x7FFFFFFF), b)
        d = np.abs(a - b)
        return k, spec_ok, int(d.max()) if d.size else 0, int((d > 0).sum())

    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as pool:
        res = list(pool.map(run, range(mud.N_CHUNKS // 2)))
    assert all(r[1] for r in res), [r[0] for r in res if not r[1]]
    assert max(r[2] for r in res) <= 1
    miss = sum(r[3] for r in res)
    assert miss <= 64, f"{miss} inputs not correctly rounded"
