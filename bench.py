#!/usr/bin/env python3
"""Throughput of the multi-hypothesis featuremetric LM solver on one MI355X.

One step = one full solve (every level, every LM pass, selection) of the
workload's frames, inputs resident in HBM before timing starts.  Default
workload (--config 3, the precision form): one synthetic frame with 3 levels
120x160x32 / 240x320x64 / 480x640x128 with bf16 maps and descriptors,
N = 16384 anchors per level, M = 1024 hypotheses within 20 m / 10 deg of the
prior, 15 LM iterations per level, gravity and laser-range priors on; beside
it the same frame through the plain FP32 solver (f32 maps) and the FP32
multi-hypothesis workload (--config 2: N = 8192, M = 256, f32).  Other
workloads: --config 1 (single hypothesis, one 120x160x32 level, latency over
many graph replays), --config 4 (64 uneven frames in one solve), --config 5
(continuous-batching serving of 16 simulated 30 Hz UAV sequences).

Prints one JSON line:
  value        point-residual (anchor x hypothesis) evaluations per second
  roofline     dominant kernel (finest-level pass kernel): the bytes one
               launch moves between L2 and HBM/MALL (rocprofv3 FETCH_SIZE +
               WRITE_SIZE, scaled by a plain copy's reading, stored in
               profiles/ for the kernel sources it was taken from) / the
               average launch duration measured here with hipEvents on the
               solver's stream; beside it the dense-equivalent gathered bytes
               (4 taps x C x bytes per element for every evaluation)
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
# wave-level VALU instructions the chip can issue per cycle: 256 CUs x 4 SIMDs,
# one wave64 instruction per SIMD every 4 cycles (16 lanes per cycle)
VALU_ISSUE_PER_CYCLE = 256 * 4 / 4
METRIC = "point-residual evals/s (GB/s vs HBM peak); p50/p99 frame latency, BF16 vs FP32"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pass_kernel_traffic.json")
TILES_FILE = os.path.join(ROOT, "paper_2606_31098_amd", "tiles_gfx950.txt")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--config", type=int, default=3, choices=[0, 1, 2, 3, 4, 5])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle sample time")
    p.add_argument("--no-bf16", action="store_true", help="config 2: skip the bf16 comparison")
    p.add_argument("--no-f32", action="store_true", help="config 3: skip the FP32 solver on the same frame")
    p.add_argument("--no-config2", action="store_true", help="config 3: skip the config-2 FP32 leg")
    p.add_argument("--frame-seed", type=int, default=0)
    p.add_argument("--no-tune", action="store_true", help="heuristic tiles instead of the autotuner")
    p.add_argument("--tune-cache", default=TILES_FILE,
                   help="tile database (read; shapes missing from it are tuned and appended)")
    p.add_argument("--write-tiles", action="store_true",
                   help="only tune the tiles of every workload shape into --tune-cache")
    p.add_argument("--serve-seconds", type=float, default=60.0, help="config 5: simulated duration")
    p.add_argument("--serve-trace", default=None, metavar="PATH",
                   help="config 5: write one JSON line per served frame (stream, sizes, arrival, admission, "
                        "completion, passes) to PATH")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run 5 plain device copies of MIB MiB (scale for the DRAM byte counters)")
    return p.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def timed_solves(ctx, dfs, steps, warmup):
    """`warmup` untimed solves, then `steps` solves bracketed by device
    synchronisations; per-step device time from events on the solver's
    stream.  Returns wall seconds, per-step ms, counters, results."""
    import torch

    from paper_2606_31098_amd import _abi as A
    from paper_2606_31098_amd.pilot import DeviceResult

    res = [DeviceResult(d.M) for d in dfs]
    fa = (A.Frame * len(dfs))(*[d.s for d in dfs])
    ra = (A.Result * len(dfs))(*[r.s for r in res])
    for _ in range(warmup):
        ctx.solve_raw(fa, len(dfs), ra)
    torch.cuda.synchronize()
    ctx.stats(reset=True)
    stream = ctx.stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        ctx.solve_raw(fa, len(dfs), ra)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [a.elapsed_time(b) for a, b in evs]
    st = ctx.stats(reset=True)
    return wall, lat, st, res


def make_context(args, flags=0):
    from paper_2606_31098_amd import _abi as A
    from paper_2606_31098_amd.pilot import Context
    tune = 0 if args.no_tune else A.FLAG_AUTOTUNE
    return Context(0, flags=flags | tune, tune_cache=args.tune_cache)


def tune(ctx, args, dfs):
    import torch
    t = time.perf_counter()
    if not args.no_tune:
        seen = set()
        for d in dfs:
            key = tuple((L.C, L.dtype, L.N.bit_length(), d.M.bit_length(), (L.H * L.W).bit_length())
                        for L in d.s.level[:d.s.n_levels])
            if key not in seen:
                seen.add(key)
                ctx.autotune(d)
        torch.cuda.synchronize()
    return time.perf_counter() - t


def roofline_leg(args, dfs, steps):
    """Profiled solves (per-launch hipEvents around every pass kernel) of
    the same workload; the finest level's pass kernel is the dominant one.
    The roof is HBM bandwidth: `achieved` is the bytes the launch moves
    between L2 and HBM/MALL, from the counter profile stored for the current
    kernel sources (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated), over
    the launch duration measured here; null when the stored profile is of
    other sources."""
    from paper_2606_31098_amd import _abi as A
    from paper_2606_31098_amd import build as B
    pctx = make_context(args, A.FLAG_PROFILE)
    tune(pctx, args, dfs)
    pwall, _, pst, _ = timed_solves(pctx, dfs, steps, 1)
    fine = max(l for l in range(A.MAX_LEVELS) if pst.timed_launches[l] > 0)
    n_launch = pst.timed_launches[fine]
    avg_ms = pst.pass_ms[fine] / n_launch
    dense_bytes = pst.pair_bytes[fine] / n_launch
    C = dfs[0].s.level[fine].C
    dt = "bf16" if dfs[0].s.level[fine].dtype == A.BF16 else "f32"
    pctx.close()
    traffic, counters, source = None, None, None
    digest = B.pass_kernel_digest()
    if os.path.exists(TRAFFIC_FILE):
        try:
            entry = json.load(open(TRAFFIC_FILE)).get(f"config{args.config}")
        except (OSError, ValueError):
            entry = None
        if entry and entry.get("pass_kernel_digest") == digest:
            traffic = entry.get("bytes_per_launch")
            source = f"{os.path.relpath(TRAFFIC_FILE, ROOT)} [config{args.config}], pass kernel sources {digest}"
            cyc, valu = entry.get("gpu_cycles_per_launch"), entry.get("valu_instructions_per_launch")
            counters = {"l2_hit_rate": entry.get("l2_hit_rate"),
                        "texture_addresser_busy": entry.get("texture_addresser_busy"),
                        "texture_data_busy": entry.get("texture_data_busy")}
            if cyc and valu:
                counters["valu_issue_frac"] = round(valu / (VALU_ISSUE_PER_CYCLE * cyc), 3)
            if entry.get("l1_bytes_per_launch"):
                counters["l1_bytes_per_launch"] = entry["l1_bytes_per_launch"]
    achieved = traffic / (avg_ms * 1e-3) / 1e9 if traffic else None
    dense_gbs = dense_bytes / (avg_ms * 1e-3) / 1e9
    if achieved is not None:
        log(f"roofline: {achieved:.1f} GB/s of HBM/MALL traffic ({achieved / HBM_PEAK_GBS:.3f} of peak), "
            f"{avg_ms:.4f} ms/launch; dense-equivalent gathers {dense_gbs:.0f} GB/s")
    else:
        log(f"roofline: no counter profile of pass kernel sources {digest} for config {args.config}; "
            f"{avg_ms:.4f} ms/launch")
    return {"bound": "hbm", "achieved": round(achieved, 1) if achieved is not None else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved is not None else None,
            "traffic": traffic, "traffic_source": source,
            "kernel": f"pass kernel C={C} {dt} (level {fine})", "launches": int(n_launch),
            "avg_launch_ms": round(avg_ms, 5), "pairs_per_launch": int(pst.pairs[fine] / n_launch),
            "dense_equivalent": {"bytes_per_launch": int(dense_bytes), "GBps": round(dense_gbs, 1),
                                 "note": "4 taps x C x element bytes for every evaluated pair; pairs whose "
                                         "projections share a cell share one gather and the maps stay in "
                                         "L2/MALL, so this exceeds every memory peak and is not a roofline"},
            "counters": counters, "profiled_ms_per_step": round(pwall * 1e3 / steps, 3)}


def cpu_leg(args, frames):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    whole hypotheses (they are independent), full N, every level; on all
    host threads, and a shorter single-thread run.  Returns the baseline
    record and the oracle's results for the sampled hypotheses."""
    import numpy as np

    import oracle
    if args.no_cpu_baseline:
        return None, None
    f = frames[0]
    Ns = [L.N for L in f.levels]

    def evals(r, k):
        ok = r["status"] != oracle.DEGENERATE
        return int(k * sum(Ns) + np.sum(r["iterations"][ok]) * float(np.mean(Ns)))

    # size the sample from a one-hypothesis probe
    t0 = time.perf_counter()
    r1 = oracle.solve(f, hyps=[0], threads=1)
    t1 = time.perf_counter() - t0
    one_thread = evals(r1, 1) / t1
    th = oracle.threads(0)
    k = int(max(1, min(f.M, args.cpu_seconds / max(t1, 1e-3) * th)))
    hyps = np.arange(k)
    t0 = time.perf_counter()
    r = oracle.solve(f, hyps=hyps)
    dt = time.perf_counter() - t0
    pairs = evals(r, k)
    log(f"cpu oracle: {pairs / dt:.4g} evals/s on {th} threads ({k} hypotheses, {dt:.1f} s); "
        f"{one_thread:.4g} evals/s on 1 thread")
    return ({"value": pairs / dt, "unit": "evals/s", "cores": int(th), "kind": "oracle",
             "sample": f"hypotheses 0..{k - 1} of frame 0 at full N, all levels; {pairs} evaluations "
                       f"(level starts + iterations x N) in {dt:.1f} s",
             "one_thread_evals_per_s": one_thread}, r)


def vs_oracle(frame, gpu, orc):
    """Pose difference of the GPU result from the oracle's on the hypotheses
    the oracle solved: over hypotheses converged (within 1 m / 1 deg of the
    truth) in both that ran every level, and how many verdicts agree.
    Hypotheses pruned in both (top-K after the pruning level) stop after that
    level's few iterations, mid-descent, so their poses are reported apart
    (`pruned_*`): the selection never reads them."""
    import numpy as np

    from synth import frames as S
    idx = orc["index"]
    tg, rg = S.pose_errors(gpu["poses"][idx], frame.gt_pose)
    to, ro = S.pose_errors(orc["poses"], frame.gt_pose)
    vg, vo = (tg <= 1.0) & (rg <= 1.0), (to <= 1.0) & (ro <= 1.0)
    pruned = (np.asarray(gpu["status"])[idx] == 4) & (np.asarray(orc["status"]) == 4)
    both = vg & vo & ~pruned
    pb = vg & vo & pruned
    dt = np.array([S.pose_errors(gpu["poses"][i], orc["poses"][k])[0][0] for k, i in enumerate(idx)])
    dr = np.array([S.pose_errors(gpu["poses"][i], orc["poses"][k])[1][0] for k, i in enumerate(idx)])
    out = {"hypotheses": int(len(idx)), "verdicts_agree": int(np.sum(vg == vo)),
           "converged_in_both": int(both.sum()),
           "max_m": float(dt[both].max()) if both.any() else None,
           "median_m": float(np.median(dt[both])) if both.any() else None,
           "max_deg": float(dr[both].max()) if both.any() else None,
           "median_deg": float(np.median(dr[both])) if both.any() else None}
    if pruned.any():
        out.update({"pruned_in_both": int(pruned.sum()), "pruned_near_truth": int(pb.sum()),
                    "pruned_max_m": float(dt[pb].max()) if pb.any() else None,
                    "pruned_max_deg": float(dr[pb].max()) if pb.any() else None})
    return out


def line(args, value, steps, warmup, ms, dtype, workload, extra):
    out = {"metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": workload}
    out.update(extra)
    return out


# ------------------------------------------------------------------ configs
def config_frames(cfg, seed):
    from synth import frames as S
    if cfg == 4:
        return S.make_batch(64, field_pool=4), "bf16"
    if cfg == 0:
        return [S.paper_shaped_frame(seed)], "f32"
    return [S.make_frame(cfg, seed)], ("bf16" if cfg == 3 else "f32")


def write_tiles(args):
    """Tune the pass-kernel tiles of every workload shape (solve configs,
    config 2 in bf16, the serving shapes) into the tile database."""
    import torch

    from paper_2606_31098_amd.pilot import Context, DeviceFrame
    from synth import frames as S
    from synth import sequences as Q
    ctx = Context(0, tune_cache=args.tune_cache)
    sets = [(c,) + config_frames(c, 0) for c in (0, 1, 2)]
    sets.append((2, config_frames(2, 0)[0], "bf16"))
    sets += [(c,) + config_frames(c, 0) for c in (3, 4)]
    sets.append((3, config_frames(3, 0)[0], "f32"))
    serve = [S.make_frame(2, 0, N=side * side // 32, M=m, level_shapes=Q.LEVELS, iters=Q.ITERS, dsm_side=side)
             for side in (128, 256, 512) for m in (64, 128, 256, 512)]
    sets.append(("serving", serve, "bf16"))
    for name, frames, dtype in sets:
        t = time.perf_counter()
        tune(ctx, args, [DeviceFrame(f, dtype=dtype) for f in frames])
        torch.cuda.synchronize()
        log(f"tiles of {name} {dtype}: {time.perf_counter() - t:.1f} s")
    ctx.close()


def bf16_inputs(frame):
    """A host copy of the frame with its maps and reference descriptors
    rounded to bf16 (round-to-nearest-even), the values the device reads."""
    import copy

    import torch
    f = copy.deepcopy(frame)
    for L in f.levels:
        L.feat = torch.as_tensor(L.feat).to(torch.bfloat16).to(torch.float32).numpy()
        L.ref = torch.as_tensor(L.ref).to(torch.bfloat16).to(torch.float32).numpy()
    return f


def solve_leg(args, frames, dtype, steps):
    """Timed solves of one workload (tiles from the database, graph replays).
    Returns the summary, the per-frame results and the device frames."""
    import numpy as np
    import torch

    from paper_2606_31098_amd.pilot import DeviceFrame
    from synth import frames as S
    dfs = [DeviceFrame(f, dtype=dtype) for f in frames]
    torch.cuda.synchronize()
    ctx = make_context(args)
    tune_s = tune(ctx, args, dfs)
    tiles = sorted({ctx.tile_choice(L.C, L.dtype, L.N, d.M, L.H * L.W) for d in dfs for L in d.s.level[:d.s.n_levels]})
    log(f"tiles ({tune_s:.1f}s): {tiles[:6]}")
    wall, lat, st, res = timed_solves(ctx, dfs, steps, args.warmup)
    pairs = sum(st.pairs)
    outs = [r.numpy() for r in res]
    errs = [S.pose_errors(o["poses"][o["best"]], f.gt_pose) for o, f in zip(outs, frames)]
    te = [e[0][0] for e in errs]
    re_ = [e[1][0] for e in errs]
    out = {"value": pairs / wall, "ms_per_step": wall * 1e3 / steps, "evals_per_step": pairs / steps,
           "gb_per_s_dense_equivalent": sum(st.pair_bytes) / wall / 1e9,
           "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)}, "tiles": tiles,
           "best_pose_error": {"median_m": float(np.median(te)), "median_deg": float(np.median(re_))},
           "graph": {"captures": st.graph_captures, "replays": st.graph_replays}}
    log(f"solve {dtype}: {out['ms_per_step']:.3f} ms/step, {out['value']:.4g} evals/s, "
        f"best-pose error median {np.median(te):.3f} m / {np.median(re_):.4f} deg")
    return out, outs, dfs, ctx


def run_solve_config(args):
    cfg = args.config
    t = time.perf_counter()
    frames, dtype = config_frames(cfg, args.frame_seed)
    log(f"generated {len(frames)} frame(s) in {time.perf_counter() - t:.1f}s")
    steps = args.steps or {0: 50, 1: 1000, 2: 50, 3: 30, 4: 20}[cfg]

    head, outs, dfs, ctx = solve_leg(args, frames, dtype, steps)
    extra = {k: head[k] for k in ("gb_per_s_dense_equivalent", "latency_ms", "evals_per_step", "tiles",
                                  "best_pose_error", "graph")}
    extra["roofline"] = roofline_leg(args, dfs, max(2, min(steps, 5)))
    if cfg == 4:
        import numpy as np
        # batch invariance: frame 0 alone equals frame 0 inside the batch
        alone = ctx.solve([dfs[0]])[0].numpy()
        extra["batch_invariance_frame0_bitwise"] = bool(
            np.array_equal(alone["poses"], outs[0]["poses"]) and np.array_equal(alone["cost"], outs[0]["cost"]))
    ctx.close()
    del dfs
    other = {}
    if cfg == 2 and not args.no_bf16:
        b, bo, bdfs, bctx = solve_leg(args, frames, "bf16", steps)
        bctx.close()
        b["solve_speedup_vs_f32"] = head["ms_per_step"] / b["ms_per_step"]
        extra["bf16_same_workload"] = b
        other["bf16"] = bo[0]
    if cfg == 3 and not args.no_f32:
        # the plain FP32 solver on the same frame (f32 maps and descriptors)
        f32, fo, fdfs, fctx = solve_leg(args, frames, "f32", steps)
        fctx.close()
        del fdfs
        f32["bf16_speedup_vs_f32"] = f32["ms_per_step"] / head["ms_per_step"]
        extra["f32_same_workload"] = f32
        log(f"bf16 vs f32 on the same frame: {f32['bf16_speedup_vs_f32']:.2f}x per solve")
    if cfg == 3 and not args.no_config2:
        c2frames, _ = config_frames(2, args.frame_seed)
        c2, _, c2dfs, c2ctx = solve_leg(args, c2frames, "f32", 50)
        c2ctx.close()
        del c2dfs
        extra["config2_f32"] = c2
    # the oracle on the inputs the headline solve read (bf16-rounded when bf16)
    ofr = [bf16_inputs(frames[0])] if dtype == "bf16" else frames[:1]
    extra["cpu_baseline"], orc = cpu_leg(args, ofr)
    if orc is not None and getattr(frames[0], "keep_top", 0) and len(orc["index"]) < frames[0].M:
        orc = None                   # a pruned subset ranks differently from the full set
    if orc is not None:
        key = f"{dtype} (oracle on the same {dtype}-valued inputs)"
        extra["vs_oracle"] = {key: vs_oracle(ofr[0], outs[0], orc)}
        if "bf16" in other:
            extra["vs_oracle"]["bf16 (oracle on the f32 inputs)"] = vs_oracle(frames[0], other["bf16"], orc)
        log(f"vs oracle: {extra['vs_oracle']}")
    names = {0: "paper-shaped context: 1 frame, N=500 anchors, 1210-hypothesis grid (+-10 m, 2 m, yaw +-1..9 deg) "
                "pruned to the top 128 after the coarse level, 3 levels 120x160 / 240x320 / 480x640 with C=32 f32, "
                "2/3/4 iterations (the paper reports 43.82 ms for its optimizer on an RTX 5090; context only)",
             1: "1 frame, 1 hypothesis, N=1024 anchors from a 64x64 DSM, one 120x160x32 f32 level, 20 LM iterations",
             2: "1 frame, 3 levels 120x160x32 / 240x320x64 / 480x640x128 f32, N=8192 anchors, M=256 hypotheses "
                "(20 m / 10 deg), 15 LM iterations per level, gravity + range priors",
             3: "precision form: 1 frame, 3 levels 120x160x32 / 240x320x64 / 480x640x128 with bf16 maps and "
                "descriptors, N=16384 anchors, M=1024 hypotheses (20 m / 10 deg), 15 LM iterations per level, "
                "gravity + range priors",
             4: "64 frames in one solve: N log-uniform 2048..32768, M in {32..512}, finest level 240x320 / 360x480 / "
                "480x640, C 32/64/128 bf16, 15 iterations per level"}
    workload = {"workload": names[cfg], "frames": len(frames),
                "hypotheses": int(sum(f.M for f in frames)), "anchors": int(sum(f.levels[0].N for f in frames))}
    return line(args, head["value"], steps, args.warmup, head["ms_per_step"], dtype, workload, extra)


class _RawFrame:
    """A pilot_frame built directly from device tensors (serving frames)."""

    def __init__(self, s, M, keep):
        self.s, self.M, self.keep = s, M, keep


def make_worlds(args):
    """Host-side data of the serving sequences, drawn in parallel worker
    processes (started fresh, before this process touches the GPU)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    from synth import sequences as Q
    n = 16
    with cf.ProcessPoolExecutor(max_workers=min(n, 16), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(Q.make_world, range(n), [args.serve_seconds] * n))


def run_serving_config(args, worlds):
    import numpy as np
    import torch

    from paper_2606_31098_amd import _abi as A
    from paper_2606_31098_amd.pilot import Context, DeviceResult
    from paper_2606_31098_amd.serving import Request, ServingLoop
    from synth import frames as S
    from synth import sequences as Q

    dev = "cuda"
    n_frames = sum(len(w.frames) for w in worlds)
    ring = Q.pyramid_ring(40, dev)
    dsm_dev = [torch.as_tensor(w.dsm.heights, device=dev) for w in worlds]
    torch.cuda.synchronize()
    budget = 24 << 30
    ctx = Context(0, max_slots=48, hbm_budget_bytes=budget, tune_cache=args.tune_cache)
    lm = dict(S.LM_DEFAULTS)
    counter = [0]
    best_poses = torch.empty((n_frames, 12), dtype=torch.float64, device=dev)
    order = {}

    def build(w, spec):
        """Device inputs of one frame (everything but the prior), made before
        the run: a frame has arrived when its inputs are on the device."""
        keep = []
        s = A.Frame()
        s.n_levels = 3
        pyr = ring[counter[0] % len(ring)]
        counter[0] += 1
        P = torch.as_tensor(spec.P, device=dev)
        x, y, z = P[:, 0].contiguous(), P[:, 1].contiguous(), P[:, 2].contiguous()
        keep += [x, y, z]
        for l, (H, W, C) in enumerate(Q.LEVELS):
            ref = Q.sample_reference(pyr[l], spec.uv[l], spec.noise_seed * 3 + l, dev)
            keep.append(ref)
            lv = s.level[l]
            lv.H, lv.W, lv.C, lv.dtype = H, W, C, A.BF16
            lv.feat = pyr[l].data_ptr()
            lv.K[:] = S.level_intrinsics(H, W)
            lv.N = int(spec.P.shape[0])
            lv.x, lv.y, lv.z = x.data_ptr(), y.data_ptr(), z.data_ptr()
            lv.ref = ref.data_ptr()
            lv.iters = Q.ITERS[l]
            lv.loss_kind, lv.loss_scale = S.default_losses(C)
        i0, j0, side = spec.crop
        crop = dsm_dev[w.seq][i0:i0 + side, j0:j0 + side].contiguous()
        keep.append(crop)
        s.dsm, s.Hd, s.Wd = crop.data_ptr(), side, side
        s.dsm_x0, s.dsm_y0, s.dsm_gsd = w.dsm.x0 + j0 * w.dsm.gsd, w.dsm.y0 + i0 * w.dsm.gsd, w.dsm.gsd
        s.use_gravity, (s.gravity_loss_kind, s.gravity_loss_scale) = 1, S.GRAVITY_LOSS
        s.g_imu[:] = list(spec.g_imu)
        s.g_world[:] = [0.0, 0.0, -1.0]
        s.lambda_imu = S.LAMBDA_IMU
        s.use_range, (s.range_loss_kind, s.range_loss_scale) = 1, S.RANGE_LOSS
        s.d_range = spec.d_range
        s.pc[:] = [(640 - 1) / 2.0, (480 - 1) / 2.0]
        s.lambda_range = S.LAMBDA_RANGE
        s.tau, s.lambda_up, s.lambda_down = lm["tau"], lm["up"], lm["down"]
        s.lambda_min_rel, s.lambda_max_rel = lm["lambda_min_rel"], lm["lambda_max_rel"]
        s.step_tol_t, s.step_tol_r, s.z_min = lm["step_tol_t"], lm["step_tol_r"], lm["z_min"]
        s.min_valid = lm["min_valid"]
        s.cost_tol = lm["cost_tol"]
        offs = torch.as_tensor(spec.offsets, device=dev)
        keep.append(offs)
        s.M = int(spec.offsets.shape[0])
        s.hyp_offsets = offs.data_ptr()
        pr = None
        if spec.init_pose is not None:            # a sequence's first frame starts from its own prior
            pr = torch.as_tensor(spec.init_pose, device=dev)[None]
            keep.append(pr)
        return s, keep, pr, DeviceResult(s.M, dev)

    def prepare_for(built):
        s, keep, pr, res = built

        def prepare(prev):
            # the stream's previous result (on the device) is this frame's prior
            if prev is None:
                assert pr is not None, "a later frame of a stream arrived without its predecessor's result"
                s.prior_poses, s.prior_best = pr.data_ptr(), None
            else:
                s.prior_poses, s.prior_best = prev.poses.data_ptr(), prev.best.data_ptr()
            return _RawFrame(s, s.M, keep + ([prev] if prev is not None else [])), res, keep
        return prepare

    t_build = time.perf_counter()
    reqs = []
    input_bytes = 0
    for w in worlds:
        for spec in w.frames:
            built = build(w, spec)
            input_bytes += sum(t.numel() * t.element_size() for t in built[1])
            reqs.append(Request(stream=w.seq, t_arrival=spec.t_arrival, prepare=prepare_for(built), tag=spec))
    torch.cuda.synchronize()
    log(f"built the inputs of {len(reqs)} frames on the device in {time.perf_counter() - t_build:.1f} s "
        f"({input_bytes / 2**30:.1f} GiB)")

    def on_complete(c):
        k = len(order)
        order[k] = c.request.tag
        best_poses[k] = c.result.poses[c.result.best.long()][0]

    loop = ServingLoop(ctx)
    ctx.stats(reset=True)
    log(f"serving {n_frames} frames of {len(worlds)} sequences over {args.serve_seconds:.0f} s")
    st = loop.run(reqs, realtime=True, on_complete=on_complete)
    counters = ctx.stats(reset=True)
    lat = [c.latency * 1e3 for c in st.completions]
    if args.serve_trace:
        with open(args.serve_trace, "w") as fh:
            for c in st.completions:
                spec = c.request.tag
                fh.write(json.dumps({"stream": spec.seq, "index": spec.index, "N": int(spec.P.shape[0]),
                                     "M": int(spec.offsets.shape[0]), "arrival": c.request.t_arrival,
                                     "admit": c.t_admit, "done": c.t_done, "passes": c.steps}) + "\n")
    bp = best_poses[:len(order)].cpu().numpy()
    te, re_ = [], []
    for k, spec in order.items():
        a, b = S.pose_errors(bp[k], spec.gt_pose)
        te.append(a[0])
        re_.append(b[0])
    te, re_ = np.array(te), np.array(re_)
    pairs = sum(counters.pairs)
    frames_per_s = len(st.completions) / st.wall
    drain = st.wall - st.last_arrival
    sustained = drain < 0.5 and st.max_queue < 4 * len(worlds)
    log(f"serving: {frames_per_s:.1f} frames/s, latency p50 {percentile(lat, 50):.2f} ms p99 "
        f"{percentile(lat, 99):.2f} ms, {pairs / st.wall:.4g} evals/s, drain {drain:.2f} s, "
        f"max queue {st.max_queue}, max active {st.max_active}, EAGAIN {st.eagain}")
    workload = {"workload": "serving: 16 simulated UAV sequences at 30 Hz (Poisson arrivals), 100-300 m altitude, "
                            "pitch 30-70 deg, DSM crops 128-512 px, N = side^2/32, M in {64..512}, 3 bf16 levels "
                            "120x160x32 / 240x320x64 / 480x640x128, 2/3/4 iterations, priors on; each frame's "
                            "inputs are on the device at its arrival time, its prior is its stream's previous result",
                "frames": len(st.completions), "sequences": len(worlds), "seconds": args.serve_seconds,
                "hbm_budget_bytes": budget, "slots": 48}
    extra = {"latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "max": max(lat)},
             "serving": {"frames_per_s": frames_per_s, "offered_frames_per_s": n_frames / args.serve_seconds,
                         "sustained": bool(sustained), "drain_s": drain, "max_queue": st.max_queue,
                         "max_active": st.max_active, "eagain": st.eagain,
                         "pose_error_m": {"median": float(np.median(te)), "p90": float(np.percentile(te, 90))},
                         "pose_error_deg": {"median": float(np.median(re_)), "p90": float(np.percentile(re_, 90))},
                         "within_1m_1deg": float(np.mean((te <= 1) & (re_ <= 1))),
                         "host_seconds": {"prepare": st.host_prepare, "admit": st.host_admit,
                                          "step": st.host_step, "poll": st.host_poll}},
             "gb_per_s_dense_equivalent": sum(counters.pair_bytes) / st.wall / 1e9,
             "roofline": None, "cpu_baseline": None}
    ctx.close()
    return line(args, pairs / st.wall, st.steps, 0, st.wall * 1e3 / max(st.steps, 1), "bf16", workload, extra)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "--gpus must be 1: the solver runs on one GPU (frames and hypothesis ranges "
                                   "would shard across GPUs with one all-gather of costs; not implemented)"}))
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 5}))
        return
    if args.write_tiles:
        write_tiles(args)
        return
    worlds = None
    if args.config == 5:
        t = time.perf_counter()
        worlds = make_worlds(args)
        log(f"generated {len(worlds)} sequences in {time.perf_counter() - t:.1f}s")
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    out = run_serving_config(args, worlds) if args.config == 5 else run_solve_config(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
