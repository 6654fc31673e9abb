"""Every binary32 bit pattern (2^32 inputs) through exp, sqrt, abs and neg on the
device, through the fused flat kernel and the C ABI, against the oracle.

The oracle's results are stored as one SHA-256 digest per chunk of 2^26 patterns
(tests/golden/unary_f32_digests.json, written by tests/golden/make_unary_digests.py,
which calls only the oracle; NaN results hashed as 0x7FC00000).  Each chunk's
patterns are generated on the device, evaluated, copied back and hashed on the host;
a differing chunk is resolved against the oracle to name its first differing
inputs.  exp, sqrt, abs and neg are correctly rounded (or exact) on both sides:
the bits must agree."""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from tests.golden import make_unary_digests as mud

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "unary_f32_digests.json")))


@pytest.fixture(scope="module")
def coot():
    import torch
    import paper_2508_11385_amd as coot
    coot.init(0)
    torch.cuda.synchronize()
    return coot


@pytest.mark.parametrize("op", ["exp", "sqrt", "abs", "neg"])
def test_all_binary32_patterns(coot, op):
    import torch
    n = 1 << mud.CHUNK_BITS
    fn = {"exp": coot.exp, "sqrt": coot.sqrt, "abs": coot.abs, "neg": lambda m: -m}[op]
    out = coot.Mat.empty(n, 1, "f32", "col")
    bad = []

    def check(k, y):
        if mud.digest(y) != GOLD["digests"][op][k]:
            from tests.test_exhaustive_unary import first_differences
            bad.append((k, first_differences(op, k, y)))

    with ThreadPoolExecutor(8) as pool:
        futs = []
        for k in range(mud.N_CHUNKS):
            v = torch.arange(k * n, (k + 1) * n, dtype=torch.int64, device="cuda")
            v = torch.where(v >= 1 << 31, v - (1 << 32), v).to(torch.int32).view(torch.float32)
            x = coot.Mat(v.view(-1, 1), "f32", "col")
            coot.eval(fn(x), out=out)
            y = out.tensor.reshape(-1).cpu().numpy()      # synchronous copy
            futs.append(pool.submit(check, k, y))
            if len(futs) > 12:                            # bound the host memory held by pending chunks
                futs.pop(0).result()
        for f in futs:
            f.result()
    assert not bad, f"{op}: {len(bad)} chunks differ, e.g. {bad[:2]}"
