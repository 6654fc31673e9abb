"""Failures forced from the host on a device: an allocator that returns NULL gives
COOT_ENOMEM and leaves nothing held; calls that take library workspace refuse a
stream under capture, while the fused element-wise evaluation is recorded into a
HIP graph and replays correctly.  Every kernel exits normally."""
import numpy as np
import pytest

import synth
from oracle import elementwise as ew
from oracle import reduce as rd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2508_11385_amd as coot
    from paper_2508_11385_amd import _coot as cc
    coot.init(0)
    yield coot, cc, torch
    cc.coot_set_allocator(None, None)


def _vec(coot, n, seed):
    x = synth.rng_for(61, seed).uniform(-1, 1, n).astype(np.float32).reshape(-1, 1)
    return x, coot.Mat.from_numpy(x, "f32", "col")


def test_allocator_returning_null_gives_enomem_and_holds_nothing(env):
    coot, cc, torch = env
    x, gx = _vec(coot, 1 << 20, 1)
    ref = rd.exact_sum(x.astype(np.float64).ravel())
    held = {}
    calls = {"alloc": 0, "null": 0}

    def alloc(n, stream):
        calls["alloc"] += 1
        if calls["alloc"] > 1:                # the first request succeeds, later ones fail
            calls["null"] += 1
            return 0
        t = torch.empty(int(n), dtype=torch.uint8, device="cuda")
        held[t.data_ptr()] = t
        return t.data_ptr()

    def dealloc(p, stream):
        held.pop(int(p))

    cc.coot_set_allocator(alloc, dealloc)
    try:
        # a full reduction takes two workspaces: the first is granted, the second is NULL
        for _ in range(2):
            with pytest.raises(cc.CootError) as e:
                coot.accu(gx)
            assert e.value.status == cc.COOT_ENOMEM
        assert calls["null"] == 2 and len(held) == 1
    finally:
        cc.coot_set_allocator(None, None)                     # returns every buffer it holds
    assert not held, f"{len(held)} buffers never returned"
    r = float(coot.accu(gx).numpy().ravel()[0])               # back on hipMalloc
    assert rd.rel_err(r, ref, rd.sum_abs(x)) <= 1e-6


def test_workspace_calls_refuse_a_capturing_stream(env):
    coot, cc, torch = env
    x, gx = _vec(coot, 100_000, 2)
    y, gy = _vec(coot, 100_000, 3)
    out = coot.Mat.empty(1, 1, "f32")
    coot.accu(gx % gy, out=out)                              # code loaded outside the capture
    torch.cuda.synchronize()
    for call in (lambda: coot.accu(gx, out=out), lambda: coot.sum(gx % gy, out=out),
                 lambda: coot.eval(gx + gy, unfused=True)):
        g = torch.cuda.CUDAGraph()
        with pytest.raises(cc.CootError) as e:
            with torch.cuda.graph(g):
                call()
        assert e.value.status == cc.COOT_EUNSUPPORTED and "capturing" in str(e.value)
        del g
    torch.cuda.synchronize()
    r = float(coot.accu(gx % gy, out=out).numpy().ravel()[0])   # the stream works afterwards
    ref = rd.exact_sum(x.astype(np.float64).ravel() * y.astype(np.float64).ravel())
    assert rd.rel_err(r, ref, rd.sum_abs(x.astype(np.float64) * y)) <= 1e-6


def test_fused_eval_is_recorded_into_a_graph_and_replays(env):
    coot, cc, torch = env
    A, B, C, D = synth.matrix_inputs(n_rows=300, n_cols=300)
    g = [coot.Mat.from_numpy(m) for m in (A, B, C, D)]
    z = coot.Mat.empty(300, 300, "f32")
    expr = 2.0 * g[0] + g[1] % g[2] - coot.trans(g[3])
    coot.eval(expr, out=z)                                   # loads the code object
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        coot.eval(expr, out=z)
    zp = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",), ("load", 3),
          ("trans",), ("sub",)]
    rng = synth.rng_for(62)
    for rep in range(4):
        # new operand values between replays (eager work and a synchronisation in between)
        mats = [rng.uniform(-1, 1, A.shape).astype(np.float32) for _ in range(4)]
        for m, v in zip(g, mats):
            m.tensor.copy_(torch.from_numpy(v))
        z.tensor.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        want = ew.evaluate(zp, mats, [2.0], "f32")
        assert np.array_equal(z.numpy(), want), rep


_TRIM_CHILD = r"""
import json, os, sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
import paper_2508_11385_amd as coot
from paper_2508_11385_amd import _coot as cc
from oracle import elementwise as ew
from tests.exact import ulp_distance
coot.init(0)
g = np.random.default_rng(7)
A = g.uniform(0.5, 2.0, (300, 7)).astype(np.float32)
B = g.uniform(-1.0, 1.0, (300, 7)).astype(np.float32)
mA, mB = coot.Mat.from_numpy(A), coot.Mat.from_numpy(B)
out = coot.Mat.empty(300, 7, "f32")
ok = True
def run(op):
    post = [("load", 0), (op,), ("load", 1), ("sub",)]
    h = cc.coot_expr_compile(post, [(cc.COOT_F32, 0)] * 2, 0)
    cc.coot_expr_eval(h, [mA.operand(), mB.operand()], [], out.operand(), None,
                      torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    good = float(np.max(ulp_distance(out.numpy(), ew.evaluate(post, [A, B], [], "f32")))) <= (1 if op in ("exp", "log") else 0)
    cc.coot_expr_release(h)   # queued work done; its module is now held by the cache alone
    return good
ops = ["neg", "abs", "sqrt", "square", "exp", "log"]
for op in ops:
    ok &= run(op)
res = {"ok": ok, "info": cc.coot_cache_info()}
res["trimmed"] = cc.coot_cache_trim()
res["info_after"] = cc.coot_cache_info()
for op in ops:                                  # evicted and unloaded modules come back from the disk cache
    ok &= run(op)
res["ok_again"] = ok
print(json.dumps(res), flush=True)
"""


def test_module_cache_eviction_and_trim_on_device(tmp_path):
    """Six modules loaded and used through a memory cache capped at two, each
    expression released after its launch: the four evicted modules wait for unloading,
    coot_cache_trim unloads them after a device synchronisation, and every expression
    evaluates correctly again afterwards (from the disk cache), in a process of its own."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, COOT_CACHE_DIR=str(tmp_path), COOT_MODULE_CACHE="2")
    env.pop("COOT_HIPRTC_EXTRA", None)
    r = subprocess.run([sys.executable, "-c", _TRIM_CHILD, root], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    o = json.loads(r.stdout.strip().splitlines()[-1])
    assert o["ok"] and o["ok_again"]
    assert o["info"] == {"modules": 2, "cap": 2, "evictions": 4, "awaiting_unload": 4}
    assert o["trimmed"] == 4
    assert o["info_after"]["awaiting_unload"] == 0
