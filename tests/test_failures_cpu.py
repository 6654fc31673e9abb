"""Failures forced from the host, without a device: a compilation error reaches the
caller as COOT_ECOMPILE with the hipRTC log and leaves nothing in the caches; a
damaged file of the on-disk code-object cache (truncated, or one byte changed) is
recompiled silently and rewritten whole."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
AXPY = [("load", 0), ("scalar", 0), ("schur",), ("load", 1), ("add",)]


@pytest.fixture(scope="module")
def cc():
    from paper_2508_11385_amd import _coot
    return _coot


# an expression no other test compiles, so that the process-wide module cache cannot
# already hold its module when this file runs after the others
UNIQUE = [("load", 0), ("load", 1), ("div",), ("scalar", 0), ("add",), ("sqrt",), ("neg",), ("square",),
          ("scalar", 1), ("sub",)]


def test_compile_error_is_reported_and_nothing_is_cached(cc, tmp_path, monkeypatch):
    monkeypatch.setenv("COOT_CACHE_DIR", str(tmp_path))
    # an include of a missing file: every module compiled under it fails
    monkeypatch.setenv("COOT_HIPRTC_EXTRA", "-include/nonexistent/coot_missing.h")
    h = cc.coot_expr_compile(UNIQUE, [(cc.COOT_F32, 0)] * 2, 2)
    before = cc.coot_stats()["compiles"]
    for _ in range(2):                       # a failed module is not remembered either
        with pytest.raises(cc.CootError) as e:
            cc.coot_expr_prepare(h, -1, rflags=cc.COOT_PF_COMPILE_ONLY)
        assert e.value.status == cc.COOT_ECOMPILE
        assert "coot_missing.h" in str(e.value) and "hipRTC compilation failed" in str(e.value)
    assert cc.coot_stats()["compiles"] == before
    assert not [f for f in os.listdir(tmp_path) if f.endswith(".co")]
    # the same request without the broken option compiles and is cached
    monkeypatch.delenv("COOT_HIPRTC_EXTRA")
    cc.coot_expr_prepare(h, -1, rflags=cc.COOT_PF_COMPILE_ONLY)
    assert cc.coot_stats()["compiles"] == before + 1
    assert len([f for f in os.listdir(tmp_path) if f.endswith(".co")]) == 1
    cc.coot_expr_release(h)


_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
from paper_2508_11385_amd import _coot as cc
h = cc.coot_expr_compile(%r, [(cc.COOT_F32, 0)] * 2, 1)
cc.coot_expr_prepare(h, -1, rflags=cc.COOT_PF_COMPILE_ONLY)
print(json.dumps(cc.coot_stats()))
""" % (AXPY,)


def _fresh_process(cache):
    """Prepare the expression in a new process (empty memory cache); its counters."""
    env = dict(os.environ, COOT_CACHE_DIR=str(cache))
    env.pop("COOT_HIPRTC_EXTRA", None)
    env.pop("COOT_NO_DISK_CACHE", None)
    r = subprocess.run([sys.executable, "-c", _CHILD, ROOT], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return json.loads(r.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("damage", ["truncate", "flip"])
def test_damaged_disk_cache_file_is_recompiled(tmp_path, damage):
    s = _fresh_process(tmp_path)
    assert (s["compiles"], s["disk_hits"]) == (1, 0)
    files = [f for f in os.listdir(tmp_path) if f.endswith(".co")]
    assert len(files) == 1
    path = os.path.join(tmp_path, files[0])
    whole = open(path, "rb").read()
    assert (_fresh_process(tmp_path)["compiles"], _fresh_process(tmp_path)["disk_hits"]) == (0, 1)
    if damage == "truncate":
        open(path, "wb").write(whole[:len(whole) // 2])
    else:                                    # one byte of the code object changed: the checksum differs
        b = bytearray(whole)
        b[len(b) - 100] ^= 0x40
        open(path, "wb").write(bytes(b))
    s = _fresh_process(tmp_path)
    assert (s["compiles"], s["disk_hits"]) == (1, 0)
    assert open(path, "rb").read() == whole  # rewritten whole
    s = _fresh_process(tmp_path)
    assert (s["compiles"], s["disk_hits"]) == (0, 1)


_LRU_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
from paper_2508_11385_amd import _coot as cc
ops = ["neg", "abs", "sqrt", "exp", "square", "log"]
def compile_one(op):
    h = cc.coot_expr_compile([("load", 0), (op,), ("load", 1), ("sub",)], [(cc.COOT_F32, 0)] * 2, 0)
    cc.coot_expr_prepare(h, -1, rflags=cc.COOT_PF_COMPILE_ONLY)
    return h
hs = [compile_one(op) for op in ops]
out = {"after_six": cc.coot_cache_info(), "stats_six": cc.coot_stats()}
cc.coot_expr_prepare(hs[0], -1, rflags=cc.COOT_PF_COMPILE_ONLY)   # held by its expression: no lookup
out["stats_held"] = cc.coot_stats()
h2 = compile_one(ops[0])                                            # evicted: back from the disk cache
out["stats_again"] = cc.coot_stats()
out["after_again"] = cc.coot_cache_info()
out["trimmed"] = cc.coot_cache_trim()                               # nothing was loaded on a device
print(json.dumps(out))
"""


def test_module_cache_evicts_least_recently_used(tmp_path):
    """A memory cache capped at 3 modules (COOT_MODULE_CACHE) over six distinct modules
    keeps the three most recent and evicts the rest; an expression keeps its own module;
    a new expression asking for an evicted module gets it from the disk cache."""
    env = dict(os.environ, COOT_CACHE_DIR=str(tmp_path), COOT_MODULE_CACHE="3")
    env.pop("COOT_HIPRTC_EXTRA", None)
    env.pop("COOT_NO_DISK_CACHE", None)
    r = subprocess.run([sys.executable, "-c", _LRU_CHILD, ROOT], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr
    o = json.loads(r.stdout.strip().splitlines()[-1])
    assert o["after_six"] == {"modules": 3, "cap": 3, "evictions": 3, "awaiting_unload": 0}
    assert o["stats_six"]["compiles"] == 6
    assert o["stats_held"] == o["stats_six"]
    assert o["stats_again"]["compiles"] == 6 and o["stats_again"]["disk_hits"] == o["stats_six"]["disk_hits"] + 1
    assert o["after_again"]["modules"] == 3 and o["after_again"]["evictions"] == 4
    assert o["trimmed"] == 0
