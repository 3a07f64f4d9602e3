#!/usr/bin/env python3
"""Throughput of the multi-hypothesis featuremetric LM solver on one MI355X.

One step = one full solve (every level, every LM pass, selection) of one
synthetic frame shaped like the paper's workload at the default size:
3 levels 120x160x32 / 240x320x64 / 480x640x128 (f32), N = 8192 anchors per
level, M = 256 hypotheses within 20 m / 10 deg of the prior, 15 LM iterations
per level, gravity and laser-range priors on.  Inputs are resident in HBM
before timing starts.

Prints one JSON line (rank 0):
  value        point-residual (anchor x hypothesis) evaluations per second
  roofline     dominant kernel (finest-level pass kernel): algorithmic
               gathered bytes (4 taps x C x 4 B per evaluation) per launch /
               average launch duration (hipEvents on the solver's stream)
  cpu_baseline the FP64 oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "point-residual evals/s (GB/s vs HBM peak); p50/p99 frame latency, BF16 vs FP32"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-hyps", type=int, default=48, help="hypotheses in the oracle sample")
    p.add_argument("--no-bf16", action="store_true")
    p.add_argument("--frame-seed", type=int, default=0)
    p.add_argument("--no-tune", action="store_true", help="heuristic tiles instead of the autotuner")
    p.add_argument("--tune-cache", default=None, help="autotune cache file (read, and appended when tuning)")
    return p.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def timed_solves(ctx, df, steps, warmup):
    """Warm-up, then `steps` solves bracketed by synchronisations; per-step
    device time from events on the solver's stream."""
    import ctypes as C

    import torch

    from paper_2606_31098_amd import _abi as A
    from paper_2606_31098_amd.pilot import DeviceResult

    res = DeviceResult(df.M)
    fa = (A.Frame * 1)(df.s)
    ra = (A.Result * 1)(res.s)
    for _ in range(warmup):
        ctx.solve_raw(fa, 1, ra)
    torch.cuda.synchronize()
    ctx.stats(reset=True)
    stream = ctx.stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        ctx.solve_raw(fa, 1, ra)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [a.elapsed_time(b) for a, b in evs]
    st = ctx.stats(reset=True)
    return wall, lat, st, res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the solver shards by frames/hypotheses across GPUs only in design)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_31098_amd import _abi as A
    from paper_2606_31098_amd.pilot import Context, DeviceFrame
    from synth import frames as S

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)

    t_gen = time.perf_counter()
    frame = S.make_frame(2, args.frame_seed)
    gen_s = time.perf_counter() - t_gen
    print(f"# generated config-2 frame in {gen_s:.1f}s", file=sys.stderr, flush=True)
    df = DeviceFrame(frame, dtype="f32")
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- timed region (graph replays)
    tune_flag = 0 if args.no_tune else A.FLAG_AUTOTUNE
    ctx = Context(0, flags=tune_flag, tune_cache=args.tune_cache)
    t_tune = time.perf_counter()
    if tune_flag:
        ctx.autotune(df)                       # tile choice per level, timed on this frame (untimed here)
        torch.cuda.synchronize()
    tune_s = time.perf_counter() - t_tune
    tiles = [ctx.tile_choice(L.C, A.F32, L.N, df.M) for L in frame.levels]
    print(f"# tiles ({tune_s:.1f}s): {tiles}", file=sys.stderr, flush=True)
    wall, lat, st, res = timed_solves(ctx, df, args.steps, args.warmup)
    pairs = sum(st.pairs)
    ms_per_step = wall * 1e3 / args.steps
    evals_per_s = pairs / wall
    gbs = sum(st.pair_bytes) / wall / 1e9
    out = res.numpy()
    te, re_ = S.pose_errors(out["poses"][out["best"]], frame.gt_pose)
    print(f"# graph: {ms_per_step:.3f} ms/step, {evals_per_s:.4g} evals/s, {gbs:.1f} GB/s algorithmic; "
          f"best={out['best']} err={te[0]:.3f} m {re_[0]:.4f} deg", file=sys.stderr, flush=True)

    # ---------------------------------------------------------------- roofline: per-launch events
    pctx = Context(0, flags=A.FLAG_PROFILE | tune_flag, tune_cache=args.tune_cache)
    if tune_flag:
        pctx.autotune(df)
    pwall, plat, pst, _ = timed_solves(pctx, df, max(3, args.steps // 4), 1)
    fine = max(l for l in range(A.MAX_LEVELS) if pst.timed_launches[l] > 0)
    n_launch = pst.timed_launches[fine]
    avg_ms = pst.pass_ms[fine] / n_launch
    bytes_per_launch = pst.pair_bytes[fine] / n_launch
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    prof_file = os.path.join(ROOT, "profiles", "pass_c128_f32_config2_traffic.json")
    if os.path.exists(prof_file):
        try:
            tj = json.load(open(prof_file))
            from paper_2606_31098_amd import build as B
            if tj.get("source_digest") == B.source_digest():
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "pass_kernel<128, f32> (finest level, 480x640x128)",
                "launches": int(n_launch), "avg_launch_ms": round(avg_ms, 5),
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "pairs_per_launch": int(pst.pairs[fine] / n_launch),
                "profiled_ms_per_step": round(pwall * 1e3 / max(3, args.steps // 4), 3)}
    print(f"# roofline: {achieved:.1f} GB/s ({achieved / HBM_PEAK_GBS:.3f} of peak), {avg_ms:.4f} ms/launch",
          file=sys.stderr, flush=True)

    # ---------------------------------------------------------------- bf16 on the same workload
    bf16 = None
    if not args.no_bf16:
        dfb = DeviceFrame(frame, dtype="bf16")
        bctx = Context(0, flags=tune_flag, tune_cache=args.tune_cache)
        if tune_flag:
            bctx.autotune(dfb)
        bwall, blat, bst, bres = timed_solves(bctx, dfb, args.steps, args.warmup)
        bout = bres.numpy()
        bte, bre = S.pose_errors(bout["poses"][bout["best"]], frame.gt_pose)
        bf16 = {"value": sum(bst.pairs) / bwall, "ms_per_step": bwall * 1e3 / args.steps,
                "latency_ms": {"p50": percentile(blat, 50), "p99": percentile(blat, 99)},
                "evals_per_step": sum(bst.pairs) / args.steps,
                "solve_speedup_vs_f32": ms_per_step / (bwall * 1e3 / args.steps),
                "best_pose_error_m": float(bte[0]), "best_pose_error_deg": float(bre[0])}
        print(f"# bf16: {bf16['ms_per_step']:.3f} ms/step ({bf16['solve_speedup_vs_f32']:.2f}x per solve)",
              file=sys.stderr, flush=True)
        bctx.close()

    # ---------------------------------------------------------------- CPU baseline (oracle sample)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        k = min(args.cpu_hyps, frame.M)
        hyps = np.arange(k)
        t0 = time.perf_counter()
        r = oracle.solve(frame, hyps=hyps)
        dt = time.perf_counter() - t0
        N = frame.levels[0].N
        ok = r["status"] != 3
        cpu_pairs = int(np.sum(N * (len(frame.levels) + r["iterations"][ok])))
        cpu = {"value": cpu_pairs / dt, "unit": "evals/s", "cores": int(oracle.threads()), "kind": "oracle",
               "sample": f"hypotheses 0..{k - 1} of the same frame, full N and all 3 levels "
                         f"({cpu_pairs} evaluations in {dt:.1f} s)"}
        print(f"# cpu oracle: {cpu['value']:.4g} evals/s on {cpu['cores']} threads", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1 frame, 3 levels 120x160x32 / 240x320x64 / 480x640x128 f32, N=8192 anchors, "
                               "M=256 hypotheses (20 m / 10 deg), 15 LM iterations per level, gravity + range priors",
                   "frames": 1, "hypotheses": 256, "anchors": 8192, "iters_per_level": 15},
        "gb_per_s_algorithmic": gbs,
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "evals_per_step": pairs / args.steps,
        "tiles": tiles,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "bf16_same_workload": bf16,
    }
    print(json.dumps(line))
    ctx.close()
    pctx.close()


if __name__ == "__main__":
    main()
