"""Learned launch-configuration tuner: timing data, training, evaluation.

The system produces its own training data: random expression signatures
(random trees of depth 1-8 over 2-5 operands, rows and cols log-uniform in
[1, 16384], element types u32 / s32 / f32 / f64, element-wise or accu) are timed
by the autotuner (coot_tune_table) over their family's configuration space; the
training set samples configurations from the training signatures' tables; a cost
model (coot_costmodel_train: MLP forward / backward / Adam kernels on the GPU)
learns log-time relative to the default configuration from the 21 features; on
held-out signatures its argmin and the exhaustive argmin are re-timed side by
side (regret = t(pick) / t(exhaustive pick) - 1).

Orchestration only: every timing, the training and the inference run through
libcoot's entry points.
"""
from __future__ import annotations

import math
import multiprocessing as mp
import os
import time

import numpy as np
import torch

import synth
from . import _coot as cc
from . import frontend

TORCH = {"f32": torch.float32, "f64": torch.float64, "u32": torch.int32, "s32": torch.int32}


def sample_signatures(n: int, seed: int, depth_hi: int = 8, dim_hi: int = 16384, p_accu: float = 0.2):
    """(TreeSpec, mode) pairs: mode -1 element-wise, 0 accu."""
    g = synth.rng_for(5, seed)
    out = []
    for _ in range(n):
        dt = ("u32", "s32", "f32", "f64")[int(g.integers(0, 4))]
        r = synth.log_uniform_int(g, 1, dim_hi)
        c = synth.log_uniform_int(g, 1, dim_hi)
        spec = synth.random_tree(g, int(g.integers(1, depth_hi + 1)), int(g.integers(2, 6)), r, c, dt)
        mode = 0 if g.random() < p_accu else -1
        out.append((spec, mode))
    return out


def _handle(spec):
    slots = [(cc.DTYPE_CODE[spec.dtype], cc.COOT_MAT)] * len(spec.slot_shapes)
    return cc.coot_expr_compile(spec.postfix, slots, len(spec.scalars))


def _fake_operands(spec):
    """Descriptors with the real shapes and an aligned placeholder address (planning only)."""
    return [cc.coot_operand(0x100000, r, c, max(1, r), cc.DTYPE_CODE[spec.dtype], cc.COOT_MAT)
            for r, c in spec.slot_shapes]


def _compile_worker(job):
    """Spawned process: compile one tuning module into the on-disk code-object cache (no device use)."""
    postfix, dtype, shapes, n_sc, mode = job
    from paper_2508_11385_amd import _coot as c2
    slots = [(c2.DTYPE_CODE[dtype], c2.COOT_MAT)] * len(shapes)
    h = c2.coot_expr_compile(postfix, slots, n_sc)
    ops = [c2.coot_operand(0x100000, r, c, max(1, r), c2.DTYPE_CODE[dtype], c2.COOT_MAT) for r, c in shapes]
    fam = c2.coot_tune_prepare(h, ops, mode)
    c2.coot_expr_release(h)
    return fam


def prepare_all(sigs, workers: int = 12, log=None):
    """Compile every signature's tuning module; returns (handles, families).

    hipRTC compilations do not overlap across threads of one process, so they run in
    `workers` spawned processes that fill the on-disk code-object cache; this process
    then loads every module from that cache.
    """
    jobs = [(s.postfix, s.dtype, s.slot_shapes, len(s.scalars), m) for s, m in sigs]
    if workers > 1 and len(jobs) > 1 and not os.environ.get("COOT_NO_DISK_CACHE"):
        t0 = time.time()
        with mp.get_context("spawn").Pool(workers) as pool:
            for k, _ in enumerate(pool.imap_unordered(_compile_worker, jobs, chunksize=4), start=1):
                if log and k % 200 == 0:
                    log(f"compiled {k}/{len(jobs)} tuning modules ({time.time() - t0:.0f} s)")
    handles = [_handle(s) for s, _ in sigs]
    fams = [cc.coot_tune_prepare(h, _fake_operands(s), m) for h, (s, m) in zip(handles, sigs)]
    return handles, fams


def _operands(spec, g):
    mats = []
    for r, c in spec.slot_shapes:
        store = torch.empty((c, r), dtype=TORCH[spec.dtype], device="cuda")
        if spec.dtype in ("f32", "f64"):
            store.uniform_(-1.0, 1.0, generator=g)
        else:
            store.random_(0, 1 << 16, generator=g)
        mats.append(frontend.Mat(store.t(), spec.dtype))
    return mats


def time_signature(h, spec, mode, cfgs, reps=5, flush=False, seed=0):
    """Median per-launch time (us) of each configuration on fresh operands of the signature's shape."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    mats = _operands(spec, g)
    r, c = spec.out_shape
    out = frontend.Mat.empty(r, c, spec.dtype) if mode < 0 else frontend.Mat.empty(1, 1, spec.dtype)
    t = cc.coot_tune_table(h, [m.operand() for m in mats], spec.scalars, out.operand(), mode, cfgs, reps, flush,
                           torch.cuda.current_stream().cuda_stream)
    del mats, out
    return np.asarray(t, np.float64)


def time_tables(sigs, handles, fams, reps=5, seed=0, log=None, what="signatures"):
    """Exhaustive timing table (configurations, times) of every signature over its family's space."""
    spaces = {0: cc.coot_tune_space(0), 1: cc.coot_tune_space(1)}
    tables = []
    t0 = time.time()
    for i, ((spec, mode), h, fam) in enumerate(zip(sigs, handles, fams)):
        cfgs = spaces[fam]
        tables.append((cfgs, time_signature(h, spec, mode, cfgs, reps=reps, seed=seed * 100003 + i)))
        if log and (i + 1) % 250 == 0:
            log(f"timed {i + 1}/{len(sigs)} {what} ({time.time() - t0:.0f} s)")
    return tables


def _valid(t):
    return np.flatnonzero(np.isfinite(t) & (t > 0))


STREAM_ELEMS = 1 << 24  # flat launches past this many elements take the library's streaming defaults
TILE_LARGE_ELEMS = 1 << 22  # tiled launches of this many elements or more default to 64 x 64 tiles


def default_index(cfgs, dtype, t=None, n=0, mode=-1):
    """What the library launches without a tuner for n elements in this mode (-1
    element-wise, else a full reduction): the default configuration, or, when the operands
    do not allow its vector width (t[k] NaN), the same with scalar accesses; a tiled
    default whose staging does not fit takes 32 x 32 tiles."""
    v = 2 if dtype == "f64" else 4
    tiled = bool(cfgs[0][4])
    if tiled:                                       # (vec, 1, 4, per CU, tile rows, tile cols)
        ts = 64 if n >= TILE_LARGE_ELEMS else 32
        want = (2, 1, 4, 8, ts, ts)
    elif n > STREAM_ELEMS:
        want = (2, 8, 4, 16, 0, 0) if mode < 0 else ((2, 4, 8, 8, 0, 0) if dtype == "f64" else (4, 4, 4, 2, 0, 0))
    else:
        want = (v, 1, 4, 4, 0, 0)
    chain = [want, (1,) + want[1:]]
    if tiled and want[4] != 32:
        chain += [(2, 1, 4, 8, 32, 32), (1, 1, 4, 8, 32, 32)]
    elif tiled:                                     # (32 x 32 staging beyond LDS: refused by the library)
        chain += [(1, 1, 4, 8, 32, 32)]
    for c in chain:
        k = cfgs.index(c)
        if t is None or np.isfinite(t[k]):
            return k
    return k


def dataset(sigs, handles, tables, configs_per_sig=None, seed=0):
    """Rows of (features, target) from the timing tables.

    Each signature contributes `configs_per_sig` sampled runnable configurations (all when
    None), always including the default one.  The target is log(time) minus log(time of
    the default configuration): the argmin only needs the ranking of a signature's
    configurations, and a common reference keeps targets comparable across signatures."""
    g = np.random.default_rng(seed)
    feats, target = [], []
    for (spec, mode), h, (cfgs, t) in zip(sigs, handles, tables):
        ok = _valid(t)
        if ok.size == 0:
            continue
        d = default_index(cfgs, spec.dtype, t, spec.out_shape[0] * spec.out_shape[1], mode)
        ref = math.log(t[d]) if d in ok else float(np.mean(np.log(t[ok])))
        if configs_per_sig is None or configs_per_sig >= ok.size:
            pick = ok
        else:
            rest = ok[ok != d]
            n = configs_per_sig - (1 if d in ok else 0)
            pick = np.sort(np.concatenate([[d] if d in ok else [], g.choice(rest, n, replace=False)]).astype(int))
        red = 0 if mode < 0 else 1
        f = cc.coot_costmodel_features(h, spec.out_shape[0], spec.out_shape[1], red, [cfgs[k] for k in pick])
        feats.append(f)
        target.append(np.log(t[pick]) - ref)
    return np.concatenate(feats).astype(np.float32), np.concatenate(target).astype(np.float32)


def he_init(seed: int, f: int = cc.N_FEATURES, h1: int = 64, h2: int = 64, n_models: int = 1):
    """He-normal initial parameters (weights N(0, 2/fan_in), biases 0) of n_models networks,
    each flat in the library's order, concatenated."""
    out = []
    for k in range(n_models):
        g = synth.rng_for(6, seed, k)
        parts = [g.normal(0, math.sqrt(2 / f), (h1, f)), np.zeros(h1), g.normal(0, math.sqrt(2 / h1), (h2, h1)),
                 np.zeros(h2), g.normal(0, math.sqrt(2 / h2), (1, h2)), np.zeros(1)]
        out.append(np.concatenate([p.ravel() for p in parts]))
    return np.concatenate(out).astype(np.float32)


COST_MODEL_MARGIN = 0.05   # coot_tune's kCostModelMargin


def picks(cm, sigs, handles, tables, margin=COST_MODEL_MARGIN):
    """Per signature: (exhaustive argmin, cost-model pick, default) as indices into its
    configuration list; the cost model ranks only the runnable configurations, and its
    argmin replaces the default only when predicted `margin` faster (0: always)."""
    out, t_pred = [], 0.0
    for (spec, mode), h, (cfgs, t) in zip(sigs, handles, tables):
        ok = _valid(t)
        exh = int(ok[np.argmin(t[ok])])
        t0 = time.perf_counter()
        k, pred = cc.coot_costmodel_predict(cm, h, spec.out_shape[0], spec.out_shape[1], 0 if mode < 0 else 1,
                                            [cfgs[i] for i in ok])
        d = default_index(cfgs, spec.dtype, t, spec.out_shape[0] * spec.out_shape[1], mode)
        # as coot_tune's cost-model policy: the default unless the network predicts a clear gain
        pos = np.flatnonzero(ok == d)
        if margin > 0 and pos.size and pred[k] > pred[pos[0]] - np.log1p(margin):
            k = int(pos[0])
        t_pred += time.perf_counter() - t0
        out.append((exh, int(ok[k]), d))
    return np.asarray(out, np.int64), t_pred / max(1, len(sigs))


def retime(sigs, handles, tables, pick_sets, reps=11, seed=0):
    """Fresh per-launch times of the picked configurations, timed side by side (interleaved
    rounds), so that no pick profits from the noise of the table it was chosen from.
    pick_sets: (n_signatures, n_policies) indices; returns times of the same shape."""
    res = np.zeros(pick_sets.shape, np.float64)
    for i, ((spec, mode), h, (cfgs, _t)) in enumerate(zip(sigs, handles, tables)):
        uniq = sorted(set(int(k) for k in pick_sets[i]))
        tt = time_signature(h, spec, mode, [cfgs[k] for k in uniq], reps=reps, seed=seed * 100003 + i)
        m = dict(zip(uniq, tt))
        res[i] = [m[int(k)] for k in pick_sets[i]]
    return res


def regrets_from_table(tables, idx):
    """t(pick) / t(best) - 1 within the exhaustive timing tables."""
    out = []
    for (cfgs, t), k in zip(tables, idx):
        out.append(t[k] / np.nanmin(t) - 1.0)
    return np.asarray(out)


def summarize(r):
    """Geometric-mean regret (geomean of the time ratios, minus 1), p90, max, share within 5%."""
    g = float(np.exp(np.mean(np.log1p(r))) - 1.0)
    return {"geomean": g, "p90": float(np.percentile(r, 90)), "max": float(np.max(r)),
            "within_5pct": float(np.mean(r <= 0.05))}


def save_tables(path, sigs, fams, handles, tables, split):
    """Timing tables and signature descriptors as plain arrays (numpy .npz, no pickled objects)."""
    meta, rows = [], []
    for i, ((spec, mode), fam, h, (cfgs, t)) in enumerate(zip(sigs, fams, handles, tables)):
        n_ops = sum(1 for it in spec.postfix if it[0] not in ("load", "scalar"))
        n_tr = sum(1 for it in spec.postfix if it[0] == "trans")
        meta.append([spec.out_shape[0], spec.out_shape[1], ("u32", "s32", "f32", "f64").index(spec.dtype), mode, fam,
                     n_ops, len(spec.slot_shapes), n_tr, split[i]])
        f = cc.coot_costmodel_features(h, spec.out_shape[0], spec.out_shape[1], 0 if mode < 0 else 1, cfgs)
        for k, c in enumerate(cfgs):
            rows.append((i, *c, t[k], *f[k]))
    rows = np.asarray(rows, np.float64)
    nc = len(tables[0][0][0]) if tables else 6   # fields of a configuration (vec, ept, waves, grid_mult, tile_r, tile_c)
    np.savez_compressed(path, meta=np.asarray(meta, np.int64), sig=rows[:, 0].astype(np.int64),
                        cfg=rows[:, 1:1 + nc].astype(np.int64), us=rows[:, 1 + nc],
                        feat=rows[:, 2 + nc:].astype(np.float32))
