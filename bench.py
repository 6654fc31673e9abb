"""Benchmark: fused-expression effective HBM bandwidth on one MI355X.

Workload (the 2-D expression workload, fp32, 4096 x 4096, column-major):
    Z = 2*A + B % C - trans(D)        (tiled kernel: trans(D) staged through LDS)
    W = exp(A) / (1 + abs(B))         (flat kernel)
    sum(2*A + B % C - trans(D), 0)    (fused per-column sums)
    sum(2*A + B % C - trans(D), 1)    (fused per-row sums)
One step runs all four.  Algorithmic bytes per step: every operand read once and
every output written once: (5 + 3 + 4 + 4) x 64 MiB + 2 x 16 KiB.
Inputs are seeded synthetic U[-1,1] data resident in HBM before timing starts.

Prints ONE JSON line: metric, value (GB/s), unit, ms_per_step, dtype, config, the
roofline of the dominant kernel (achieved and peak bandwidth, their ratio, HBM traffic
from the committed counter summary) and the CPU oracle's rate on a sample.  --gpus
above 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 4096
MIB64 = N * N * 4
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--cpu-cols", type=int, default=4096, help="columns of the problem the CPU oracle is timed on")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-other-configs", action="store_true",
                   help="skip the other workloads (axpy+dot, fp64 step, integers, 2^28 reductions, batch)")
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_tile_Z_4096_f32.json"))
    p.add_argument("--workload", default="expr4096", choices=["expr4096", "batch", "tuner", "suite"],
                   help="expr4096: the fused 2-D expression step (default); batch: 10,000 small expressions")
    p.add_argument("--batch-n", type=int, default=10_000)
    p.add_argument("--tune", default="exhaustive", choices=["exhaustive", "none"],
                   help="launch configurations of Z and W: the exhaustive autotuner's pick (before the timed "
                        "region; the step with the library defaults is timed too) or the library defaults")
    p.add_argument("--z-cfg", default="", help="launch configuration vec,ept,waves,grid_mult[,tile_r,tile_c] for Z "
                                              "(default: the autotuner's pick)")
    p.add_argument("--w-cfg", default="", help="launch configuration vec,ept,waves,grid_mult for W "
                                              "(default: the autotuner's pick)")
    p.add_argument("--batch-fused-sample", type=int, default=500,
                   help="expressions timed with the plain fused kernel, one launch each")
    p.add_argument("--tuner-train", type=int, default=1350, help="training signatures (~50,000 timings)")
    p.add_argument("--tuner-test", type=int, default=2000, help="held-out signatures (timed exhaustively)")
    p.add_argument("--tuner-cfgs", type=int, default=50, help="configurations timed per training signature")
    p.add_argument("--tuner-epochs", type=int, default=200)
    p.add_argument("--tuner-reps", type=int, default=5, help="timing rounds per configuration")
    p.add_argument("--tuner-models", type=int, default=5, help="networks in the cost-model ensemble")
    p.add_argument("--tuner-dump", default="", help="write the timing tables here (.npz)")
    p.add_argument("--tuner-out", default=os.path.join(tempfile.gettempdir(), "costmodel_mi355x.bin"),
                   help="where the trained cost model is saved")
    p.add_argument("--tuner-workers", type=int, default=14, help="processes compiling tuning modules")
    p.add_argument("--profile-kernels", action="store_true",
                   help="run the copy probe and each kernel of one step 3 times, print their names, exit")
    p.add_argument("--batch-parts", default="",
                   help="with --workload batch --profile-kernels: split the workload into its expressions "
                        "with a trans() (2-D tiles) and the rest (flat chunks), build each as a batch of its "
                        "own with this configuration (vec,ept,waves,grid_mult) and launch the 2-D one 3 times, "
                        "then the flat one")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding across GPUs "
              "is designed but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2508_11385_amd as coot
    from paper_2508_11385_amd import _coot as cc
    import synth

    coot.init(0)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "tuner":
        return bench_tuner(args)
    if args.workload == "suite":
        return bench_suite(args)
    dev = torch.device("cuda:0")
    A, B, C, D = synth.matrix_inputs(N, "f32")
    gA, gB, gC, gD = (coot.Mat.from_numpy(m) for m in (A, B, C, D))
    Zout = coot.Mat.empty(N, N, "f32")
    Wout = coot.Mat.empty(N, N, "f32")
    s0 = coot.Mat.empty(1, N, "f32", "row")
    s1 = coot.Mat.empty(N, 1, "f32", "col")

    zexpr = 2.0 * gA + gB % gC - coot.trans(gD)
    wexpr = coot.exp(gA) / (1.0 + coot.abs(gB))
    zf, wf = coot.flatten(zexpr), coot.flatten(wexpr)

    def handles(flags):
        return coot.frontend.compiled(zf, flags), coot.frontend.compiled(wf, flags)

    zops = [m.operand() for m in zf.mats]
    wops = [m.operand() for m in wf.mats]
    zo, wo, s0o, s1o = Zout.operand(), Wout.operand(), s0.operand(), s1.operand()
    stream = torch.cuda.current_stream().cuda_stream

    bytes_step = 16 * MIB64 + 2 * N * 4
    fused = handles(0)
    unfused = handles(cc.COOT_CF_UNFUSED)

    # launch configurations of the step's statements: the ones given on the command line,
    # else the project's autotuner (exhaustive over the family's space: repeated-call
    # timings, near-ties broken by cache-cold ones), run once before any timed region
    cfgs = {"Z": None, "W": None, "S0": None, "S1": None}
    for k, v in (("Z", args.z_cfg), ("W", args.w_cfg)):
        if v:
            cfgs[k] = tuple(int(x) for x in v.split(","))
    t0 = time.perf_counter()
    if args.tune == "exhaustive":
        if not cfgs["Z"]:
            cfgs["Z"] = cc.coot_tune(fused[0], zops, zf.scalars, zo, -1, 1, stream=stream)[0]
        if not cfgs["W"]:
            cfgs["W"] = cc.coot_tune(fused[1], wops, wf.scalars, wo, -1, 1, stream=stream)[0]
        cfgs["S0"] = cc.coot_tune(fused[0], zops, zf.scalars, s0o, cc.COOT_RED_SUM, 1, stream=stream, dim=0)[0]
        cfgs["S1"] = cc.coot_tune(fused[0], zops, zf.scalars, s1o, cc.COOT_RED_SUM, 1, stream=stream, dim=1)[0]
    t_tune = time.perf_counter() - t0
    tuned = any(cfgs.values())

    def step(hz, hw, zc=None, wc=None, s0c=None, s1c=None):
        cc.coot_expr_eval(hz, zops, zf.scalars, zo, zc, stream)
        cc.coot_expr_eval(hw, wops, wf.scalars, wo, wc, stream)
        cc.coot_reduce(hz, zops, zf.scalars, cc.COOT_RED_SUM, 0, 0, s0o, s0c, stream)
        cc.coot_reduce(hz, zops, zf.scalars, cc.COOT_RED_SUM, 1, 0, s1o, s1c, stream)

    # copy probe: out = A through the flat family, 64 MiB read + 64 MiB written
    copy_flat = coot.flatten(gA + 0.0)
    copy_flat.postfix = [("load", 0)]
    copy_flat.scalars = []
    hcopy = coot.frontend.compiled(copy_flat)
    copy_out = coot.Mat.empty(N, N, "f32")
    cops, cout = [gA.operand()], copy_out.operand()

    def copy():
        cc.coot_expr_eval(hcopy, cops, [], cout, None, stream)

    if args.profile_kernels:
        for _ in range(3):
            copy()
        for _ in range(3):
            step(*fused, cfgs["Z"], cfgs["W"], cfgs["S0"], cfgs["S1"])
        # Z under every tile shape and vector width the autotuner can pick (its counters do
        # not depend on the launch's workgroups per CU)
        zvariants = {}
        for tr, tc in sorted({(c[4], c[5]) for c in cc.coot_tune_space(1)}):
            for vec in (1, 2, 4):
                if vec <= tr * tc // 256:
                    zc = (vec, 0, 0, 0, tr, tc)
                    for _ in range(3):
                        cc.coot_expr_eval(fused[0], zops, zf.scalars, zo, zc, stream)
                    zvariants[cc.coot_expr_kernel_name(fused[0], cfg=zc)] = zc
        torch.cuda.synchronize()
        names = {"copy": cc.coot_expr_kernel_name(hcopy), "Z": cc.coot_expr_kernel_name(fused[0], cfg=cfgs["Z"]),
                 "W": cc.coot_expr_kernel_name(fused[1], cfg=cfgs["W"]),
                 "sumZ0": cc.coot_expr_kernel_name(fused[0], cc.COOT_RED_SUM, 0, cfg=cfgs["S0"]),
                 "sumZ1": cc.coot_expr_kernel_name(fused[0], cc.COOT_RED_SUM, 1, cfg=cfgs["S1"])}
        print(json.dumps({"profiled_kernels": names, "Z_variants": sorted(zvariants), "copy_bytes": 2 * MIB64,
                          "Z_bytes": 5 * MIB64, "launches_each": 3}), flush=True)
        return

    for _ in range(3):
        copy()
    torch.cuda.synchronize()
    cev = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        copy()
        e1.record()
        cev.append((e0, e1))
    torch.cuda.synchronize()
    copy_ms = sorted(a.elapsed_time(b) for a, b in cev)[len(cev) // 2]
    copy_gbs = 2 * MIB64 / (copy_ms * 1e-3) / 1e9

    def run(h, steps, warmup, zc=None, wc=None, z_events=None, s0c=None, s1c=None):
        for _ in range(warmup):
            step(*h, zc, wc, s0c, s1c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            if z_events is not None:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record()
                cc.coot_expr_eval(h[0], zops, zf.scalars, zo, zc, stream)
                ev1.record()
                z_events.append((ev0, ev1))
                cc.coot_expr_eval(h[1], wops, wf.scalars, wo, wc, stream)
                cc.coot_reduce(h[0], zops, zf.scalars, cc.COOT_RED_SUM, 0, 0, s0o, s0c, stream)
                cc.coot_reduce(h[0], zops, zf.scalars, cc.COOT_RED_SUM, 1, 0, s1o, s1c, stream)
            else:
                step(*h, zc, wc, s0c, s1c)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # the chosen and the default configurations are timed in alternating blocks of steps, so
    # that clock and temperature drift over the run affects both alike; no events are
    # recorded inside these steps (a pair of event records costs several microseconds)
    tc = (cfgs["Z"], cfgs["W"])
    ts = {"s0c": cfgs["S0"], "s1c": cfgs["S1"]}
    for _ in range(args.warmup):
        step(*fused, *tc, cfgs["S0"], cfgs["S1"])
        step(*fused)
    blocks = 4 if args.steps >= 4 else 1
    per = [args.steps // blocks + (1 if k < args.steps % blocks else 0) for k in range(blocks)]
    t_fused = t_default = 0.0
    for n in per:
        t_fused += run(fused, n, 0, *tc, **ts) * n
        if tuned:
            t_default += run(fused, n, 0) * n
    t_fused /= args.steps
    t_default = t_default / args.steps if tuned else t_fused
    # the Z kernel's launch duration for the roofline: the same steps again, with HIP events
    # around each Z launch on its stream
    z_events = []
    run(fused, args.steps, 0, *tc, z_events, **ts)
    z_ms = sum(a.elapsed_time(b) for a, b in z_events) / len(z_events)
    t_unfused = run(unfused, max(3, args.steps // 4), 2)

    # cache-cold protocol: before each measured kernel a 512 MiB read evicts L2 and the
    # Infinity Cache; HIP events bracket that kernel (or the statement's kernels) only;
    # median of `reps` after 3 warm-ups
    def cold(fn, reps=20):
        ts = []
        for i in range(reps + 3):
            cc.coot_flush_caches(stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if i >= 3:
                ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2] * 1e-3

    hz, hw = fused
    parts = {
        "Z": (lambda: cc.coot_expr_eval(hz, zops, zf.scalars, zo, cfgs["Z"], stream), 5 * MIB64),
        "W": (lambda: cc.coot_expr_eval(hw, wops, wf.scalars, wo, cfgs["W"], stream), 3 * MIB64),
        "sumZ0": (lambda: cc.coot_reduce(hz, zops, zf.scalars, cc.COOT_RED_SUM, 0, 0, s0o, cfgs["S0"], stream),
                  4 * MIB64 + N * 4),
        "sumZ1": (lambda: cc.coot_reduce(hz, zops, zf.scalars, cc.COOT_RED_SUM, 1, 0, s1o, cfgs["S1"], stream),
                  4 * MIB64 + N * 4),
    }
    cold_s = {k: cold(fn) for k, (fn, nb) in parts.items()}

    # streaming protocol: Z back to back over four copies of its operands and output (1.25 GiB
    # in rotation, far beyond the 256 MB Infinity Cache), so every launch reads HBM, in the
    # steady state of repeated launches (no flush in between); HIP events around 32 launches
    zsets = [(zops, zo)]
    keep = []
    for _ in range(3):
        cp = [coot.Mat(m.tensor.clone(), "f32") for m in zf.mats]
        zc_out = coot.Mat.empty(N, N, "f32")
        keep.append((cp, zc_out))
        zsets.append(([m.operand() for m in cp], zc_out.operand()))
    for _ in range(2):
        for ops_k, out_k in zsets:
            cc.coot_expr_eval(hz, ops_k, zf.scalars, out_k, cfgs["Z"], stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(8):
        for ops_k, out_k in zsets:
            cc.coot_expr_eval(hz, ops_k, zf.scalars, out_k, cfgs["Z"], stream)
    e1.record()
    torch.cuda.synchronize()
    z_stream_s = e0.elapsed_time(e1) * 1e-3 / (8 * len(zsets))
    z_stream_gbs = 5 * MIB64 / z_stream_s / 1e9

    # the same protocol for flat reference kernels moving the same streams as Z (four 64 MiB
    # reads and one write: A + B - C + D; its accu, four reads) and for a copy (one read, one
    # write): what HBM sustains for each stream pattern on this machine
    def streamed(launch_k):
        for _ in range(2):
            for k in range(len(zsets)):
                launch_k(k)
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(8):
            for k in range(len(zsets)):
                launch_k(k)
        a1.record()
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) * 1e-3 / (8 * len(zsets))

    mats_k = [list(zf.mats)] + [cp for cp, _ in keep]
    zsets_ops = [ops_k for ops_k, _ in zsets]
    outs_k = [zo] + [o.operand() for _, o in keep]
    ref_flat = coot.flatten(zf.mats[0] + zf.mats[1] - zf.mats[2] + zf.mats[3])
    href = coot.frontend.compiled(ref_flat)
    rops = [[m.operand() for m in ms] for ms in mats_k]
    racc_m = coot.Mat.empty(1, 1, "f32")       # kept alive while its operand is used
    racc = racc_m.operand()
    cops_k = [[ms[0].operand()] for ms in mats_k]
    # each reference at its fastest flat configuration under this protocol (every vec, ept,
    # waves and 1-16 workgroups per CU, through the tuning module: one compilation)
    flat_space = cc.coot_tune_space(0) + [(v, e, w, 1, 0, 0) for v in (1, 2, 4) for e in (1, 2, 4, 8)
                                          for w in (1, 2, 4, 8)]
    references = {}
    for name, nb, h_ref, ops_k, mode, out_of in (
            ("copy_1read_1write", 2 * MIB64, hcopy, cops_k, -1, lambda k: outs_k[k]),
            ("flat_4reads_1write", 5 * MIB64, href, rops, -1, lambda k: outs_k[k]),
            ("accu_4reads", 4 * MIB64, href, rops, cc.COOT_RED_ACCU, lambda k: racc)):
        best = None
        for c in flat_space:
            try:
                t = streamed(lambda k: cc.coot_tune_launch(h_ref, ops_k[k], [], out_of(k), mode, c, stream))
            except cc.CootError:
                continue
            if best is None or t < best[0]:
                best = (t, c)
        t, c = best
        references[name] = {"us": round(t * 1e6, 2), "GBps": round(nb / t / 1e9, 1),
                            "frac": round(nb / t / 1e9 / PEAK_HBM_GBS, 3), "cfg": list(c[:4])}
    # Z itself at its fastest tiled configuration under this protocol
    zbest = None
    for c in cc.coot_tune_space(1):
        try:
            t = streamed(lambda k: cc.coot_tune_launch(hz, zsets_ops[k], zf.scalars, outs_k[k], -1, c, stream))
        except cc.CootError:
            continue
        if zbest is None or t < zbest[0]:
            zbest = (t, c)
    del keep, zsets, mats_k, rops, cops_k, racc_m
    cold_step = sum(cold_s.values())
    hzu, hwu = unfused
    uparts = {
        "Z": lambda: cc.coot_expr_eval(hzu, zops, zf.scalars, zo, None, stream),
        "W": lambda: cc.coot_expr_eval(hwu, wops, wf.scalars, wo, None, stream),
        "sumZ0": lambda: cc.coot_reduce(hzu, zops, zf.scalars, cc.COOT_RED_SUM, 0, 0, s0o, None, stream),
        "sumZ1": lambda: cc.coot_reduce(hzu, zops, zf.scalars, cc.COOT_RED_SUM, 1, 0, s1o, None, stream),
    }
    cold_unfused = sum(cold(fn, 10) for fn in uparts.values())
    # unfused bytes per step: every operator reads its operands and writes a temporary
    # (Z: 13, W: 9, each fused sum: Z's 13 + 1) x 64 MiB, against 16 x 64 MiB fused
    byte_ceiling = (13 + 9 + 14 + 14) / 16

    value = bytes_step / t_fused / 1e9
    z_gbs = 5 * MIB64 / (z_ms * 1e-3) / 1e9
    zname = cc.coot_expr_kernel_name(fused[0], cfg=cfgs["Z"])
    traffic = measured_traffic(args.traffic_json, zname)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, B, C, D, args.cpu_cols)
    others = None
    if not args.no_other_configs:
        del gA, gB, gC, gD, Zout, Wout, copy_out, zexpr, wexpr, zf, wf, copy_flat, zops, wops, cops
        torch.cuda.empty_cache()
        others = other_configs(args)

    out = {
        "metric": "fused-expr effective HBM GB/s (% of peak); speedup vs unfused per-op kernels",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_fused * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded U[-1,1] fp32 operands, resident in HBM",
        "config": {"workload": "Z=2*A+B%C-trans(D), W=exp(A)/(1+abs(B)), sum(Z,0), sum(Z,1) fused; "
                               "fp32 4096x4096 column-major",
                   "n_rows": N, "n_cols": N, "bytes_per_step": bytes_step},
        "pct_of_peak": round(100 * value / PEAK_HBM_GBS, 1),
        "copy_probe_gbs": round(copy_gbs, 1),
        "pct_of_copy_probe": round(100 * value / copy_gbs, 1),
        "kernels": {"copy": cc.coot_expr_kernel_name(hcopy), "Z": zname,
                    "W": cc.coot_expr_kernel_name(fused[1], cfg=cfgs["W"]),
                    "sumZ0": cc.coot_expr_kernel_name(fused[0], cc.COOT_RED_SUM, 0, cfg=cfgs["S0"]),
                    "sumZ1": cc.coot_expr_kernel_name(fused[0], cc.COOT_RED_SUM, 1, cfg=cfgs["S1"])},
        "launch_cfgs": {"Z": cfgs["Z"], "W": cfgs["W"], "sumZ0": cfgs["S0"], "sumZ1": cfgs["S1"],
                        "fields": "vec, ept, waves, grid_mult, tile_r, tile_c",
                        "chosen_by": ("exhaustive autotuner before timing" +
                                      ("; given on the command line: " + ", ".join(
                                          k for k, v in (("Z", args.z_cfg), ("W", args.w_cfg)) if v)
                                       if (args.z_cfg or args.w_cfg) else ""))
                        if args.tune == "exhaustive" else ("given" if tuned else "library defaults"),
                        "tuning_s": round(t_tune, 2)},
        "default_cfg_ms_per_step": round(t_default * 1e3, 4),
        "unfused_ms_per_step": round(t_unfused * 1e3, 4),
        "speedup_vs_unfused": round(t_unfused / t_fused, 2),
        "speedup_byte_ceiling": byte_ceiling,
        "unfused_comparator": "one kernel and one temporary per operator, plain stores (temporaries stay "
                              "in L2 / the Infinity Cache for the next operator), steps back to back",
        "cold": {
            "protocol": "512 MiB read before each measured kernel (evicts L2 and the Infinity Cache), HIP "
                        "events around that kernel (a sum: its two stages) only, median of 20",
            "ms_per_step": round(cold_step * 1e3, 4),
            "GBps": round(bytes_step / cold_step / 1e9, 1),
            "pct_of_peak": round(100 * bytes_step / cold_step / 1e9 / PEAK_HBM_GBS, 1),
            "kernels": {k: {"us": round(cold_s[k] * 1e6, 2), "GBps": round(nb / cold_s[k] / 1e9, 1),
                            "frac": round(nb / cold_s[k] / 1e9 / PEAK_HBM_GBS, 3)} for k, (fn, nb) in parts.items()},
            "unfused_ms_per_step": round(cold_unfused * 1e3, 4),
            "speedup_vs_unfused": round(cold_unfused / cold_step, 2),
        },
        "roofline": {"bound": "hbm", "kernel": zname,
                     "achieved": round(z_stream_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(z_stream_gbs / PEAK_HBM_GBS, 3), "traffic": traffic,
                     "avg_kernel_us": round(z_stream_s * 1e6, 2), "algorithmic_bytes": 5 * MIB64,
                     "measured": "HIP events on the launch stream around 32 back-to-back Z launches over 4 copies "
                                 "of its operands and output (1.25 GiB in rotation: every launch reads HBM, no "
                                 "Infinity Cache reuse)",
                     "of_same_stream_reference": round(references["flat_4reads_1write"]["us"] / (z_stream_s * 1e6), 3),
                     "streaming_references": references,
                     "best_tiled_streaming": {"us": round(zbest[0] * 1e6, 2), "cfg": list(zbest[1]),
                                              "frac": round(5 * MIB64 / zbest[0] / 1e9 / PEAK_HBM_GBS, 3)},
                     "in_step": {"us": round(z_ms * 1e3, 2), "frac": round(z_gbs / PEAK_HBM_GBS, 3),
                                 "note": "HIP events around each Z launch of the timed steps: A, B, C, D are "
                                         "re-read by the step's other kernels, partly from the Infinity Cache"},
                     "cold": {"us": round(cold_s["Z"] * 1e6, 2),
                              "frac": round(5 * MIB64 / cold_s["Z"] / 1e9 / PEAK_HBM_GBS, 3),
                              "note": "one launch after a 512 MiB flush, median of 20"}},
        "cpu_baseline": cpu,
        "other_configs": others,
    }
    print(json.dumps(out), flush=True)


def other_configs(args):
    """The other workloads the method is specified on, each at its full size, GPU time by HIP
    events (inputs resident in HBM): axpy then dot on 1e6 fp32 (two statements, and one pass),
    the 4096 x 4096 step in fp64 (library defaults, and autotuned), u32 (A+B)%C and s32 A-3*B on 8192 x 8192, compensated
    accu and norm over 2^28 lognormal fp32 values, and 10,000 small expressions as one
    autotuned batch launch.  Bytes are algorithmic (operands read once, results written
    once); `cold` times single launches after a 512 MiB cache flush (median of 10)."""
    import numpy as np
    import torch
    import paper_2508_11385_amd as coot
    from paper_2508_11385_amd import _coot as cc
    import synth

    stream = torch.cuda.current_stream().cuda_stream

    def warm_us(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    def cold_us(fn, reps=10):
        ts = []
        for i in range(reps + 2):
            cc.coot_flush_caches(stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if i >= 2:
                ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2] * 1e3

    def autotuned(nbytes, e, out, mode=-1, reps=10):
        """The same call with coot_tune's exhaustive pick (element-wise or accu)."""
        f = coot.flatten(e)
        h = coot.frontend.compiled(f)
        ops, oo = [m.operand() for m in f.mats], out.operand()
        t0 = time.perf_counter()
        pick = cc.coot_tune(h, ops, f.scalars, oo, mode, 1, stream=stream)[0]
        t_tune = time.perf_counter() - t0
        if mode < 0:
            fn = lambda: cc.coot_expr_eval(h, ops, f.scalars, oo, pick, stream)  # noqa: E731
        else:
            fn = lambda: cc.coot_reduce(h, ops, f.scalars, mode, -1, 0, oo, pick, stream)  # noqa: E731
        r = entry(nbytes, fn, reps=reps)
        r.update({"pick": pick, "tuning_s": round(t_tune, 2)})
        return r

    def entry(nbytes, fn, cold=True, reps=20):
        us = warm_us(fn, reps)
        r = {"us": round(us, 2), "GBps": round(nbytes / us / 1e3, 1),
             "frac": round(nbytes / us / 1e3 / PEAK_HBM_GBS, 3), "bytes": nbytes}
        if cold:
            uc = cold_us(fn)
            r.update({"us_cold": round(uc, 2), "GBps_cold": round(nbytes / uc / 1e3, 1),
                      "frac_cold": round(nbytes / uc / 1e3 / PEAK_HBM_GBS, 3)})
        return r

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    res = {}
    # axpy y = 2.5 x + y in place, then accu(x % y) with the new y, on 1e6 fp32
    x, y = synth.axpy_inputs()
    gx, gy = coot.Mat.from_numpy(x, kind="col"), coot.Mat.from_numpy(y, kind="col")
    n = x.shape[0]

    def two_statements():
        coot.eval(2.5 * gx + gy, out=gy)
        coot.accu(gx % gy)

    # statements built once and called repeatedly (the front end keeps each expression
    # object's flattened form and argument arrays)
    axpy, dotx = 2.5 * gx + gy, gx % gy
    d1 = coot.Mat.empty(1, 1, "f32")

    def two_statements():
        coot.eval(axpy, out=gy)
        coot.accu(dotx, out=d1)

    res["axpy_then_dot_1e6_f32"] = {
        "two_statements": entry(20 * n, two_statements, cold=False, reps=200),
        "one_pass": entry(12 * n, lambda: coot.eval_reduce(axpy, gy, dotx, res=d1), cold=False, reps=200),
        "note": "4 + 4 MB operands stay in the Infinity Cache between calls: latency-bound, not a "
                "bandwidth workload"}
    log(f"axpy+dot {res['axpy_then_dot_1e6_f32']}")
    # host cost of one call on a cached expression: calls queued back to back on a tiny
    # operand, wall time per call with the GPU work far shorter than the host's
    t1 = coot.Mat.from_numpy(np.ones((256, 1), np.float32), kind="col")
    t2 = coot.Mat.empty(256, 1, "f32", "col")
    te = 2.0 * t1 + t1
    tflat = coot.flatten(te)
    th = coot.frontend.compiled(tflat)
    tops = cc._arr(cc.coot_operand, [m.operand() for m in tflat.mats])
    tsc = cc._arr(cc.C.c_double, tflat.scalars)
    tout = t2.operand()

    def host_us(fn, reps=2000):
        for _ in range(50):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        t = time.perf_counter() - t0
        torch.cuda.synchronize()
        return t / reps * 1e6

    res["host_us_per_call"] = {
        "abi_eval": round(host_us(lambda: cc.lib.coot_expr_eval(th, tops, tsc, cc.C.byref(tout), None, stream)), 2),
        "frontend_eval": round(host_us(lambda: coot.eval(te, out=t2)), 2),
        "frontend_accu": round(host_us(lambda: coot.accu(te, out=d1)), 2),
        "frontend_eval_new_tree": round(host_us(lambda: coot.eval(2.0 * t1 + t1, out=t2)), 2),
        "note": "wall time per call of calls queued back to back (256-element operands): the library "
                "call alone (ctypes), and through the front end on a cached expression object, "
                "and with the tree built anew each call"}
    log(f"host {res['host_us_per_call']}")
    del gx, gy, t1, t2

    # the 2-D step in fp64
    A, B, C, D = synth.matrix_inputs(N, "f64")
    gA, gB, gC, gD = (coot.Mat.from_numpy(m) for m in (A, B, C, D))
    del A, B, C, D
    Z = 2.0 * gA + gB % gC - coot.trans(gD)
    W = coot.exp(gA) / (1.0 + coot.abs(gB))
    oz, ow = coot.Mat.empty(N, N, "f64"), coot.Mat.empty(N, N, "f64")
    s0, s1 = coot.Mat.empty(1, N, "f64", "row"), coot.Mat.empty(N, 1, "f64", "col")

    def step64():
        coot.eval(Z, out=oz)
        coot.eval(W, out=ow)
        coot.sum(Z, 0, out=s0)
        coot.sum(Z, 1, out=s1)

    res["step_4096_f64"] = entry(2 * (16 * MIB64 + 2 * N * 4), step64, reps=10)
    # the same step with the autotuner's picks (exhaustive, as for the fp32 step)
    zf, wf = coot.flatten(Z), coot.flatten(W)
    hz, hw = coot.frontend.compiled(zf), coot.frontend.compiled(wf)
    zo, wo_, s0o, s1o = oz.operand(), ow.operand(), s0.operand(), s1.operand()
    zops, wops = [m.operand() for m in zf.mats], [m.operand() for m in wf.mats]
    t0 = time.perf_counter()
    pz = cc.coot_tune(hz, zops, zf.scalars, zo, -1, 1, stream=stream)[0]
    pw = cc.coot_tune(hw, wops, wf.scalars, wo_, -1, 1, stream=stream)[0]
    p0 = cc.coot_tune(hz, zops, zf.scalars, s0o, cc.COOT_RED_SUM, 1, stream=stream, dim=0)[0]
    p1 = cc.coot_tune(hz, zops, zf.scalars, s1o, cc.COOT_RED_SUM, 1, stream=stream, dim=1)[0]
    t_tune = time.perf_counter() - t0

    def step64_tuned():
        cc.coot_expr_eval(hz, zops, zf.scalars, zo, pz, stream)
        cc.coot_expr_eval(hw, wops, wf.scalars, wo_, pw, stream)
        cc.coot_reduce(hz, zops, zf.scalars, cc.COOT_RED_SUM, 0, 0, s0o, p0, stream)
        cc.coot_reduce(hz, zops, zf.scalars, cc.COOT_RED_SUM, 1, 0, s1o, p1, stream)

    t = entry(2 * (16 * MIB64 + 2 * N * 4), step64_tuned, reps=10)
    t.update({"picks": {"Z": pz, "W": pw, "sumZ0": p0, "sumZ1": p1}, "tuning_s": round(t_tune, 2)})
    res["step_4096_f64"]["autotuned"] = t
    del gA, gB, gC, gD, Z, W, oz, ow, s0, s1, zf, wf
    torch.cuda.empty_cache()
    log(f"fp64 step {res['step_4096_f64']}")

    # integers on 8192 x 8192
    M = 8192
    Ai, Bi, Ci = synth.int_inputs(M, "u32")
    gA, gB, gC = (coot.Mat.from_numpy(m) for m in (Ai, Bi, Ci))
    del Ai, Bi, Ci
    o = coot.Mat.empty(M, M, "u32")
    eu = (gA + gB) % gC
    res["u32_(A+B)%C_8192"] = entry(4 * 4 * M * M, lambda: coot.eval(eu, out=o), reps=10)
    res["u32_(A+B)%C_8192"]["autotuned"] = autotuned(4 * 4 * M * M, eu, o)
    del gA, gB, gC, o, eu
    As, Bs = synth.int_inputs(M, "s32_full")
    gA, gB = coot.Mat.from_numpy(As), coot.Mat.from_numpy(Bs)
    del As, Bs
    o = coot.Mat.empty(M, M, "s32")
    es = gA - 3 * gB
    res["s32_A-3B_8192"] = entry(3 * 4 * M * M, lambda: coot.eval(es, out=o), reps=10)
    res["s32_A-3B_8192"]["autotuned"] = autotuned(3 * 4 * M * M, es, o)
    del gA, gB, o, es
    torch.cuda.empty_cache()
    log("integers done")

    # compensated accu and norm over 2^28 lognormal(0, 4) fp32 values with random signs
    h = synth.hard_reduction_inputs()
    gh = coot.Mat.from_numpy(h, kind="col")
    del h
    nb = 4 * (1 << 28)
    o1 = coot.Mat.empty(1, 1, "f32")
    res["accu_2^28_f32"] = entry(nb, lambda: coot.accu(gh, out=o1), reps=10)
    res["accu_2^28_f32"]["autotuned"] = autotuned(nb, gh, o1, cc.COOT_RED_ACCU)
    res["norm_2^28_f32"] = entry(nb, lambda: coot.norm(gh, out=o1), reps=10)
    res["accu_plain_2^28_f32"] = entry(nb, lambda: coot.accu(gh, plain=True, out=o1), cold=False, reps=10)
    del gh, o1
    torch.cuda.empty_cache()
    log("2^28 reductions done")

    # 10,000 small expressions in one autotuned graph launch
    specs = synth.batch_workload(args.batch_n, seed=3)
    g = synth.rng_for(3, 1)
    exprs = [_tree(coot, spec, [coot.Mat.from_numpy(o) for o in synth.operands_for(spec, g)]) for spec in specs]
    b = coot.Batch([(e, None) for e in exprs])
    t0 = time.perf_counter()
    b.tune()
    t_tune = time.perf_counter() - t0
    info = b.info()
    r = entry(info["bytes"], b.launch, reps=20)
    r.update({"expressions": info["n_exprs"], "tiles": info["n_tiles"], "tuning_s": round(t_tune, 2)})
    res["batch_10000_f32"] = r
    del b, exprs
    torch.cuda.empty_cache()
    log(f"batch {r}")
    res["learned_tuner"] = "bench.py --workload tuner (trains on ~50,000 autotuner timings: minutes)"
    return res


def _tree(coot, spec, mats):
    st = []
    for it in spec.postfix:
        if it[0] == "load":
            st.append(mats[it[1]])
        elif it[0] == "scalar":
            st.append(coot.Scalar(spec.scalars[it[1]]))
        elif it[0] in ("add", "sub", "schur", "div"):
            b, a = st.pop(), st.pop()
            st.append(coot.Node(it[0], [a, b]))
        else:
            st.append(coot.Node(it[0], [st.pop()]))
    return st[0]


def bench_batch(args):
    """10,000 independent fp32 expressions (random trees, depth 1-6, 2-5 operands, rows and cols
    log-uniform in [8, 512]) in one graph-captured persistent launch, default and autotuned,
    against one launch per expression."""
    import torch
    import paper_2508_11385_amd as coot
    import synth

    t0 = time.perf_counter()
    specs = synth.batch_workload(args.batch_n, seed=3)
    g = synth.rng_for(3, 1)
    exprs = []
    for spec in specs:
        mats = [coot.Mat.from_numpy(o) for o in synth.operands_for(spec, g)]
        exprs.append(_tree(coot, spec, mats))
    t_gen = time.perf_counter() - t0
    if args.profile_kernels and args.batch_parts:
        cfg = tuple(int(x) for x in args.batch_parts.split(","))
        has_t = [any(it[0] == "trans" for it in coot.flatten(e).postfix) for e in exprs]
        parts = {"2d": coot.Batch([(e, None) for e, t in zip(exprs, has_t) if t], cfg=cfg),
                 "flat": coot.Batch([(e, None) for e, t in zip(exprs, has_t) if not t], cfg=cfg)}
        for p in parts.values():         # one batch after the other: a trace tells them apart by order
            for _ in range(3):
                p.launch()
            torch.cuda.synchronize()
        print(json.dumps({"profiled": "batch parts x3", "cfg": cfg,
                          "info": {k: p.info() for k, p in parts.items()}}), flush=True)
        return
    t0 = time.perf_counter()
    b = coot.Batch([(e, None) for e in exprs])
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    info = b.info()
    if args.profile_kernels:
        for _ in range(3):
            b.launch()
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "batch graph x3", "info": info}), flush=True)
        return

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2] * 1e-3

    t_default = timed(b.launch, max(5, args.steps))
    t_each = timed(b.launch_each, 3)
    # the plain fused kernel, one launch per expression, on a sample of the workload (its
    # kernels compiled ahead of time, outside the timing, like the batch's bytecode)
    import ctypes
    from paper_2508_11385_amd import _coot as cc
    ns = min(args.batch_fused_sample, len(exprs))
    t0 = time.perf_counter()
    flats = coot.precompile(exprs[:ns])
    t_pre = time.perf_counter() - t0
    stream = torch.cuda.current_stream().cuda_stream
    calls = []
    for k, f in enumerate(flats):
        ops = (cc.coot_operand * len(f.mats))(*[m.operand() for m in f.mats])
        sc = (ctypes.c_double * max(1, len(f.scalars)))(*f.scalars)
        calls.append((coot.frontend.compiled(f), ops, sc, b.outs[k].operand()))

    def fused_each():
        for h, ops, sc, out in calls:
            st = cc.lib.coot_expr_eval(h, ops, sc, ctypes.byref(out), None, stream)
            if st != cc.COOT_OK:
                raise RuntimeError(cc.lib.coot_last_error().decode())

    t_fused_each = timed(fused_each, 3)
    bsub = coot.Batch([(e, None) for e in exprs[:ns]])
    bsub.tune()
    t_bsub = timed(bsub.launch, max(5, args.steps))
    t0 = time.perf_counter()
    cfg, tuned_us = b.tune()
    t_tune = time.perf_counter() - t0
    t_tuned = timed(b.launch, max(5, args.steps))
    info2 = b.info()
    gbs = info["bytes"] / t_tuned / 1e9
    out = {
        "metric": "batched fused-expr effective HBM GB/s; speedup vs per-expression launches",
        "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": max(5, args.steps),
        "higher_is_better": True, "dtype": "f32", "data": "synthetic: seeded random trees, U[-1,1] operands",
        "config": {"workload": f"{info['n_exprs']} random fp32 expressions, depth 1-6, 2-5 operands, "
                               "rows/cols log-uniform [8,512]", "tiles": info2["n_tiles"],
                   "algorithmic_bytes": info["bytes"]},
        "ms_tuned": round(t_tuned * 1e3, 4), "ms_default": round(t_default * 1e3, 4),
        "ms_per_expression_launches": round(t_each * 1e3, 3),
        "speedup_vs_per_expression_launches": round(t_each / t_tuned, 1),
        "fused_kernel_per_expression_sample": {
            "expressions": ns, "ms_fused_kernel_launches": round(t_fused_each * 1e3, 3),
            "ms_batch": round(t_bsub * 1e3, 4), "speedup": round(t_fused_each / t_bsub, 1),
            "precompile_s": round(t_pre, 1)},
        "tuned_cfg": {"flat_part": {"tile": info2["tile"], "elements_per_thread": 4 * info2["g"],
                                    "grid": info2["grid"], "vec": cfg[0]},
                      "2d_part": {"tile": info2["tile_2d"], "elements_per_thread": 4 * info2["g_2d"],
                                  "grid": info2["grid_2d"]},
                      "flat_tiles": info2["flat_tiles"], "parts_side_by_side": bool(info2["concurrent"])},
        "default_cfg": {"flat_part": {"tile": info["tile"], "grid": info["grid"]},
                        "2d_part": {"tile": info["tile_2d"], "grid": info["grid_2d"]},
                        "parts_side_by_side": bool(info["concurrent"])},
        "vec4_exprs": info2["vec4_exprs"], "pct_of_peak": round(100 * gbs / PEAK_HBM_GBS, 1),
        "tuning_s": round(t_tune, 2), "create_s": round(t_create, 2), "generate_s": round(t_gen, 1),
    }
    print(json.dumps(out), flush=True)


def bench_suite(args):
    """The other workloads of the method at their full sizes, GPU time by HIP events (inputs
    resident in HBM): axpy + dot on 1e6 fp32, the 4096 x 4096 step in fp64, the u32 / s32
    8192 x 8192 expressions, and accu / norm / plain accu over 2^28 lognormal fp32 values."""
    import numpy as np
    import torch
    import paper_2508_11385_amd as coot
    import synth

    def gpu_us(fn, reps=10):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    from paper_2508_11385_amd import _coot as cc
    stream = torch.cuda.current_stream().cuda_stream

    def tuned_cfg(e, out, mode):
        """the exhaustive autotuner's pick for this expression (mode -1 element-wise, else accu)"""
        f = coot.flatten(e)
        h = coot.frontend.compiled(f)
        return cc.coot_tune(h, [m.operand() for m in f.mats], f.scalars, out.operand(), mode, 1, stream=stream)[0]

    def both(name, fn, e, out, mode, nbytes):
        """time with the library defaults and with the autotuned configuration"""
        us_d = gpu_us(lambda: fn(None))
        t0 = time.perf_counter()
        cfg = tuned_cfg(e, out, mode)
        t_tune = time.perf_counter() - t0
        us_t = gpu_us(lambda: fn(cfg))
        res[name] = {"us": round(us_d, 1), "GBps": round(nbytes / us_d / 1e3, 1),
                     "us_tuned": round(us_t, 1), "GBps_tuned": round(nbytes / us_t / 1e3, 1),
                     "tuned_cfg": list(cfg), "tuning_s": round(t_tune, 2)}
        return cfg

    res = {}
    # axpy y = 2.5 x + y in place, then accu(x % y) (the dot pattern) on 1e6 fp32
    x, y = synth.axpy_inputs()
    gx, gy = coot.Mat.from_numpy(x, kind="col"), coot.Mat.from_numpy(y, kind="col")
    n = x.shape[0]

    def axpy_dot():
        coot.eval(2.5 * gx + gy, out=gy)
        return coot.accu(gx % gy)
    us = gpu_us(axpy_dot, 50)
    res["axpy_then_dot_1e6_f32"] = {"us": round(us, 2), "GBps": round(20 * n / us / 1e3, 1),
                                    "note": "two launches + one stage-2; latency-bound at this size"}
    # the same two statements as one pass (reads x and y once, writes y once: 12 bytes per element)
    us = gpu_us(lambda: coot.eval_reduce(2.5 * gx + gy, gy, gx % gy), 50)
    res["axpy_dot_one_pass_1e6_f32"] = {"us": round(us, 2), "GBps": round(12 * n / us / 1e3, 1),
                                        "note": "one launch + one stage-2 (coot_expr_eval_reduce)"}
    del gx, gy
    log(f"axpy+dot: {res['axpy_then_dot_1e6_f32']}")
    # the 2-D step in fp64
    A, B, C, D = synth.matrix_inputs(N, "f64")
    gA, gB, gC, gD = (coot.Mat.from_numpy(m) for m in (A, B, C, D))
    del A, B, C, D
    Z = 2.0 * gA + gB % gC - coot.trans(gD)
    W = coot.exp(gA) / (1.0 + coot.abs(gB))
    oz, ow = coot.Mat.empty(N, N, "f64"), coot.Mat.empty(N, N, "f64")

    def step64():
        coot.eval(Z, out=oz)
        coot.eval(W, out=ow)
        coot.sum(Z, 0)
        coot.sum(Z, 1)
    us = gpu_us(step64)
    res["step_4096_f64"] = {"us": round(us, 1), "GBps": round(2 * (16 * MIB64 + 2 * N * 4) / us / 1e3, 1)}
    del gA, gB, gC, gD, Z, W, oz, ow
    torch.cuda.empty_cache()
    log(f"fp64 step: {res['step_4096_f64']}")
    # the same step on 16-bit storage (binary32 arithmetic, every operator rounded to the type)
    for dt in ("f16", "bf16"):
        A, B, C, D = synth.matrix_inputs(N, dt)
        gA, gB, gC, gD = (coot.Mat.from_numpy(m, dtype=dt) for m in (A, B, C, D))
        del A, B, C, D
        Z = 2.0 * gA + gB % gC - coot.trans(gD)
        W = coot.exp(gA) / (1.0 + coot.abs(gB))
        oz, ow = coot.Mat.empty(N, N, dt), coot.Mat.empty(N, N, dt)

        def step16():
            coot.eval(Z, out=oz)
            coot.eval(W, out=ow)
            coot.sum(Z, 0)
            coot.sum(Z, 1)
        us = gpu_us(step16)
        nb = (16 * MIB64 + 2 * N * 4) // 2
        res[f"step_4096_{dt}"] = {"us": round(us, 1), "GBps": round(nb / us / 1e3, 1),
                                  "elements_per_ns": round(16 * N * N / us / 1e3, 1)}
        del gA, gB, gC, gD, Z, W, oz, ow
        torch.cuda.empty_cache()
        log(f"{dt} step: {res[f'step_4096_{dt}']}")
    # statistics on the fp32 Z (algorithmic bytes: one read of the four operands; mean and
    # variance are one pass each)
    A, B, C, D = synth.matrix_inputs(N, "f32")
    gA, gB, gC, gD = (coot.Mat.from_numpy(m, dtype="f32") for m in (A, B, C, D))
    del A, B, C, D
    Z = 2.0 * gA + gB % gC - coot.trans(gD)
    nb = 4 * 4 * N * N
    for name, fn in (("mean_dim0", lambda: coot.mean(Z, dim=0)), ("mean_dim1", lambda: coot.mean(Z, dim=1)),
                     ("var_dim0", lambda: coot.var(Z, dim=0)), ("var_dim1", lambda: coot.var(Z, dim=1)),
                     ("var_all", lambda: coot.var(Z))):
        us = gpu_us(fn)
        res[f"{name}_Z_4096_f32"] = {"us": round(us, 1), "GBps": round(nb / us / 1e3, 1)}
    del gA, gB, gC, gD, Z
    torch.cuda.empty_cache()
    log("statistics done")
    # integers on 8192 x 8192
    M = 8192
    Ai, Bi, Ci = synth.int_inputs(M, "u32")
    gA, gB, gC = (coot.Mat.from_numpy(m) for m in (Ai, Bi, Ci))
    o = coot.Mat.empty(M, M, "u32")
    eu = (gA + gB) % gC
    both("u32_(A+B)%C_8192", lambda cfg: coot.eval(eu, out=o, cfg=cfg), eu, o, -1, 4 * 4 * M * M)
    del gA, gB, gC, o, eu
    As, Bs = synth.int_inputs(M, "s32_full")
    gA, gB = coot.Mat.from_numpy(As), coot.Mat.from_numpy(Bs)
    o = coot.Mat.empty(M, M, "s32")
    es = gA - 3 * gB
    both("s32_A-3B_8192", lambda cfg: coot.eval(es, out=o, cfg=cfg), es, o, -1, 3 * 4 * M * M)
    del gA, gB, o, es
    torch.cuda.empty_cache()
    log("integers done")
    # reductions over 2^28 lognormal(0, 4) fp32 values with random signs
    h = synth.hard_reduction_inputs()
    gh = coot.Mat.from_numpy(h, kind="col")
    del h
    o1 = coot.Mat.empty(1, 1, "f32")
    nb = 4 * (1 << 28)
    both("accu_2^28_f32", lambda c: coot.accu(gh, cfg=c), gh, o1, cc.COOT_RED_ACCU, nb)
    # (the autotuner covers element-wise evaluation and accu: norm and the plain sum run
    # with the library defaults)
    for name, fn in (("norm", lambda: coot.norm(gh)), ("accu_plain", lambda: coot.accu(gh, plain=True)),
                     ("max", lambda: coot.max(gh)), ("min", lambda: coot.min(gh)), ("mean", lambda: coot.mean(gh)),
                     ("norm1", lambda: coot.norm1(gh)), ("norm_inf", lambda: coot.norm_inf(gh)),
                     ("var", lambda: coot.var(gh))):
        us = gpu_us(fn)
        res[f"{name}_2^28_f32"] = {"us": round(us, 1), "GBps": round(nb / us / 1e3, 1)}
    out = {"metric": "throughput of the other workloads (GB/s of algorithmic bytes)", "value": None,
           "unit": "GB/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic, seeded, resident in HBM",
           "config": {"workload": "axpy+dot 1e6 f32; 4096^2 step f64, f16, bf16; mean / var along dims and "
                              "var of Z 4096^2 f32; u32/s32 8192^2; "
                              "accu/norm/min/max/mean/norm1/norm_inf/var 2^28 f32"},
           "results": res}
    print(json.dumps(out), flush=True)


def bench_tuner(args):
    """Learned tuner: timing data generated by the autotuner, MLP trained on the GPU, regret of its
    argmin against exhaustive autotuning on held-out signatures."""
    import numpy as np
    from paper_2508_11385_amd import _coot as cc
    from paper_2508_11385_amd import tuner

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    os.environ.setdefault("COOT_CACHE_DIR", "/tmp/coot_cache")   # shared by the compile workers
    # held-out signatures come from a seed that played no part in choosing the library's
    # default configurations (those were fitted on the tables of seeds 1 and 2)
    train = tuner.sample_signatures(args.tuner_train, seed=1)
    test = tuner.sample_signatures(args.tuner_test, seed=3)
    t0 = time.perf_counter()
    h_tr, f_tr = tuner.prepare_all(train, workers=args.tuner_workers, log=log)
    h_te, f_te = tuner.prepare_all(test, workers=args.tuner_workers, log=log)
    t_compile = time.perf_counter() - t0
    log(f"compiled {len(train) + len(test)} tuning modules in {t_compile:.0f} s")
    t0 = time.perf_counter()
    tab_tr = tuner.time_tables(train, h_tr, f_tr, reps=args.tuner_reps, seed=11, log=log, what="training signatures")
    t_train_tab = time.perf_counter() - t0
    t0 = time.perf_counter()
    tab_te = tuner.time_tables(test, h_te, f_te, reps=args.tuner_reps, seed=12, log=log, what="held-out signatures")
    t_exh = time.perf_counter() - t0
    X, y = tuner.dataset(train, h_tr, tab_tr, configs_per_sig=args.tuner_cfgs, seed=13)
    n_exh = int(sum(np.isfinite(t).sum() for _, t in tab_te))
    log(f"{len(y)} training timings; {n_exh} held-out timings in {t_exh:.0f} s")
    if args.tuner_dump:
        tuner.save_tables(args.tuner_dump, train + test, f_tr + f_te, h_tr + h_te, tab_tr + tab_te,
                          [0] * len(train) + [1] * len(test))
    init = tuner.he_init(7, n_models=args.tuner_models)
    t0 = time.perf_counter()
    cm, losses = cc.coot_costmodel_train(X, y, np.ones(len(y), np.float32), init, 64, 64, args.tuner_epochs, 256, 7,
                                         1e-3, n_models=args.tuner_models)
    t_fit = time.perf_counter() - t0
    P, t_pred = tuner.picks(cm, test, h_te, tab_te)            # the library's cost-model policy
    Pa, _ = tuner.picks(cm, test, h_te, tab_te, margin=0.0)     # the network's argmin alone
    cm0, _ = cc.coot_costmodel_train(X, y, np.ones(len(y), np.float32), init, 64, 64, 0, 256, 7, 1e-3,
                                     n_models=args.tuner_models)
    P0, _ = tuner.picks(cm0, test, h_te, tab_te, margin=0.0)
    # columns: exhaustive, MLP policy, default configuration, untrained MLP argmin, MLP argmin
    sets = np.stack([P[:, 0], P[:, 1], P[:, 2], P0[:, 1], Pa[:, 1]], 1)
    t0 = time.perf_counter()
    fresh = tuner.retime(test, h_te, tab_te, sets, reps=11, seed=14)
    t_retime = time.perf_counter() - t0
    if args.tuner_dump:
        base = os.path.splitext(args.tuner_dump)[0]
        np.savez_compressed(base + "_picks.npz", picks=sets, fresh_us=fresh)
    os.makedirs(os.path.dirname(args.tuner_out), exist_ok=True)
    cc.coot_costmodel_save(cm, args.tuner_out)
    cols = ((1, "mlp"), (2, "default_config"), (3, "untrained_mlp"), (4, "mlp_argmin"))
    reg = {name: tuner.summarize(fresh[:, j] / fresh[:, 0] - 1.0) for j, name in cols}
    in_table = {name: tuner.summarize(tuner.regrets_from_table(tab_te, sets[:, j])) for j, name in cols}
    rnd = lambda d: {k: round(v, 4) for k, v in d.items()}

    # 95 % bootstrap intervals of the re-timed geomean regrets (signatures resampled), and
    # the slices of the held-out set: small outputs, reductions, fp64, the tiled family
    rng = np.random.default_rng(15)
    lr = np.log(fresh[:, 1:] / fresh[:, :1])   # log time ratios: mlp, default, untrained, mlp argmin
    boots = np.exp(np.stack([lr[rng.integers(0, len(lr), len(lr))].mean(0) for _ in range(2000)])) - 1.0
    ci = {name: [round(float(np.percentile(boots[:, j], 2.5)), 4), round(float(np.percentile(boots[:, j], 97.5)), 4)]
          for j, name in enumerate(("mlp", "default_config", "untrained_mlp", "mlp_argmin"))}
    gain = np.exp(np.stack([(lr[idx, 1] - lr[idx, 0]).mean() for idx in
                            (rng.integers(0, len(lr), len(lr)) for _ in range(2000))]))
    elems = np.array([s.out_shape[0] * s.out_shape[1] for s, _ in test])
    slices = {"outputs < 2^16 elements": elems < (1 << 16), "outputs >= 2^20 elements": elems >= (1 << 20),
              "accu": np.array([m == 0 for _, m in test]), "fp64": np.array([s.dtype == "f64" for s, _ in test]),
              "tiled family": np.array(f_te) == 1}
    by_slice = {}
    for name, msk in slices.items():
        if msk.sum() == 0:
            continue
        g = np.exp(lr[msk].mean(0)) - 1.0
        by_slice[name] = {"signatures": int(msk.sum()), "mlp": round(float(g[0]), 4),
                          "default_config": round(float(g[1]), 4), "mlp_argmin": round(float(g[3]), 4)}
    out = {
        "metric": "learned tuner: geomean regret of MLP-chosen launch configs vs exhaustive autotune",
        "value": round(100 * reg["mlp"]["geomean"], 2), "unit": "% regret", "higher_is_better": False, "n_gpus": 1,
        "dtype": "f32 (MLP); u32/s32/f32/f64 expressions",
        "data": "synthetic: random trees depth 1-8, rows/cols log-uniform [1,16384], timings generated on this GPU",
        "config": {"workload": "learned launch-configuration tuner", "train_signatures": len(train),
                   "train_timings": int(len(y)), "test_signatures": len(test), "test_timings": n_exh,
                   "epochs": args.tuner_epochs, "hidden": [64, 64], "ensemble": args.tuner_models,
                   "reps": args.tuner_reps},
        "regret_definition": "t(pick)/t(exhaustive argmin) - 1, both picks re-timed side by side (11 interleaved "
                             "rounds of back-to-back launches) after the exhaustive table chose its argmin",
        "mlp": rnd(reg["mlp"]), "default_config": rnd(reg["default_config"]),
        "untrained_mlp": rnd(reg["untrained_mlp"]), "mlp_argmin": rnd(reg["mlp_argmin"]),
        "mlp_policy": f"the network's argmin where it predicts at least {tuner.COST_MODEL_MARGIN:.0%} over the "
                      "library default, else the default (mlp_argmin: the argmin always)",
        "regret_within_exhaustive_table": {k: rnd(v) for k, v in in_table.items()},
        "geomean_95pct_bootstrap": ci,
        "default_over_mlp_time_ratio_95pct": [round(float(np.percentile(gain, 2.5)), 4),
                                              round(float(np.percentile(gain, 97.5)), 4)],
        "by_slice": by_slice,
        "final_train_loss": round(float(losses[-1]), 4), "first_train_loss": round(float(losses[0]), 4),
        "mlp_predict_us_per_signature": round(1e6 * t_pred, 1),
        "exhaustive_tuning_s_per_signature": round(t_exh / len(test), 4),
        "compile_s": round(t_compile, 1), "train_tables_s": round(t_train_tab, 1), "fit_s": round(t_fit, 2),
        "retime_s": round(t_retime, 1),
    }
    print(json.dumps(out), flush=True)


def kernel_source_hash() -> str:
    """sha256 over the device headers and the code generator (what decides the kernel's traffic)."""
    import hashlib
    h = hashlib.sha256()
    dev = os.path.join(ROOT, "paper_2508_11385_amd", "csrc", "device")
    for f in sorted(os.listdir(dev)):
        if f.endswith(".h"):
            h.update(open(os.path.join(dev, f), "rb").read())
    h.update(open(os.path.join(ROOT, "paper_2508_11385_amd", "csrc", "codegen.cpp"), "rb").read())
    return h.hexdigest()


def measured_traffic(path, kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE summary
    (every variant of the Z kernel is recorded there), or None when the kernel is not in it
    or its sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return k.get("bytes_per_launch") if k else None


def cpu_baseline(A, B, C, D, ncols):
    """The oracle, as it stands, on the first `ncols` columns of the same step."""
    import numpy as np
    from oracle import elementwise as ew
    from oracle import reduce as rd
    zp = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",), ("load", 3),
          ("trans",), ("sub",)]
    wp = [("load", 0), ("exp",), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]
    a, b, c, d = A[:, :ncols], B[:, :ncols], C[:, :ncols], D[:ncols, :]
    t0 = time.perf_counter()
    rounds = 0
    while True:   # whole steps until about 10 s of CPU work
        ew.evaluate(zp, [a, b, c, d], [2.0], "f32")
        ew.evaluate(wp, [a, b], [1.0], "f32")
        Z2 = ew.evaluate(zp, [a, b, c, d], [2.0], "f32")
        [rd.to_float(q) for q in rd.sum_dim(Z2, 0, "f32")]
        Z3 = ew.evaluate(zp, [a, b, c, d], [2.0], "f32")
        [rd.to_float(q) for q in rd.sum_dim(Z3, 1, "f32")]
        rounds += 1
        if time.perf_counter() - t0 >= 10.0:
            break
    dt = time.perf_counter() - t0
    nbytes = 16 * N * ncols * 4 * rounds
    return {"value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the same four expressions on columns 0..{ncols - 1} of the 4096x4096 operands "
                      f"({ncols / N:.3f} of one step), {rounds} rounds in {dt:.1f} s, numpy single-threaded "
                      f"(1 of {os.cpu_count()} host cores)"}


if __name__ == "__main__":
    main()
