"""Serving (continuous batching) against the oracle and against solves.

Frames shaped like the serving workload (DSM crops of 128-512 samples,
N = side^2 / 32 anchors, 64-512 hypotheses generated on the device around
the stream's previous result, bf16 pyramids 120x160x32 / 240x320x64 /
480x640x128, 2/3/4 iterations) go through the request loop with the
benchmark's tile database; a sample of them is solved again by the oracle on
the same (bf16-exact) inputs and the same hypotheses."""
import os

import numpy as np
import pytest
import torch

import oracle
from synth import frames as S
from synth import sequences as Q
from tests.gpu_common import BF16_TOL_DEG, BF16_TOL_M, POSE_TOL_DEG, POSE_TOL_M, compare_solutions, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TILES = os.path.join(ROOT, "paper_2606_31098_amd", "tiles_gfx950.txt")


def host_frame(world, spec, pyr_host, refs_host):
    """The frame's inputs as a synth Frame (maps and descriptors are the
    bf16 values the device holds, widened to f32)."""
    i0, j0, side = spec.crop
    dsm = S.Dsm(heights=np.ascontiguousarray(world.dsm.heights[i0:i0 + side, j0:j0 + side]),
                x0=world.dsm.x0 + j0 * world.dsm.gsd, y0=world.dsm.y0 + i0 * world.dsm.gsd, gsd=world.dsm.gsd)
    levels = []
    for l, (H, W, C) in enumerate(Q.LEVELS):
        levels.append(S.Level(H=H, W=W, C=C, feat=pyr_host[l], K=S.level_intrinsics(H, W),
                              x=spec.P[:, 0].copy(), y=spec.P[:, 1].copy(), z=spec.P[:, 2].copy(),
                              ref=refs_host[l], iters=Q.ITERS[l], loss=S.default_losses(C)))
    M = spec.offsets.shape[0]
    return S.Frame(levels=levels, poses=np.zeros((M, 12)), dsm=dsm, g_imu=spec.g_imu, d_range=spec.d_range,
                   pc=((640 - 1) / 2.0, (480 - 1) / 2.0), gt_pose=spec.gt_pose)


def _floor_log2(n):
    return max(int(n), 1).bit_length() - 1


def _serving_inputs(n_seq=3, seconds=0.2, iters=None):
    worlds = [Q.make_world(s, seconds) for s in range(n_seq)]
    ring = Q.pyramid_ring(3, "cuda")
    ring_host = [[m.float().cpu().numpy() for m in pyr] for pyr in ring]
    frames = {}
    k = 0
    for w in worlds:
        for spec in w.frames:
            pyr = ring[k % len(ring)]
            refs = [Q.sample_reference(pyr[l], spec.uv[l], spec.noise_seed * 3 + l) for l in range(3)]
            hf = host_frame(w, spec, ring_host[k % len(ring)], [r.float().cpu().numpy() for r in refs])
            if iters is not None:
                for L, it in zip(hf.levels, iters):
                    L.iters = it
            frames[(w.seq, spec.index)] = (hf, spec)
            k += 1
    torch.cuda.synchronize()
    return worlds, frames


def _serve(frames, tune_cache):
    """Every frame through the request loop (all arrive at once; each stream
    runs its frames in order, a frame's prior being its predecessor's result,
    and the streams share the device).  Returns the results by frame."""
    from paper_2606_31098_amd.pilot import Context, DeviceFrame, DeviceResult
    from paper_2606_31098_amd.serving import Request, ServingLoop
    reqs = []
    for key, (hf, spec) in sorted(frames.items()):
        def prepare(prev, hf=hf, spec=spec):
            if prev is None:
                prior, best = torch.as_tensor(spec.init_pose[None], device="cuda"), None
            else:
                prior, best = prev.poses, prev.best
            df = DeviceFrame(hf, dtype="bf16", prior=prior, prior_best=best, hyp_offsets=spec.offsets)
            return df, DeviceResult(df.M), [prior]
        reqs.append(Request(stream=key[0], t_arrival=0.0, prepare=prepare, tag=key))
    ctx = Context(0, max_slots=16, tune_cache=tune_cache)
    done = {}
    st = ServingLoop(ctx).run(reqs, realtime=False, on_complete=lambda c: done.__setitem__(c.request.tag, c.result))
    assert len(st.completions) == len(reqs)
    assert st.max_active > 1                        # frames overlapped on the device
    out = {key: r.numpy() for key, r in done.items()}
    ctx.close()
    return out


def _prior_of(frames, res, key):
    hf, spec = frames[key]
    seq, idx = key
    if idx == 0:
        return spec.init_pose
    prev = res[(seq, idx - 1)]
    return prev["poses"][prev["best"]]


def _against_oracle(frames, res, keys, tol_m, tol_deg, per_frame=32):
    for key in keys:
        hf, spec = frames[key]
        prior = _prior_of(frames, res, key)
        hf.poses = np.stack([S.hypothesis(prior, *o) for o in spec.offsets])
        hyps = np.arange(0, hf.M, max(1, hf.M // per_frame))
        say(f"frame {key}: N={hf.levels[0].N} M={hf.M}, oracle on {len(hyps)} hypotheses")
        orc = oracle.solve(hf, hyps=hyps, threads=0)
        gpu = {k: (v[hyps] if isinstance(v, np.ndarray) and v.shape[:1] == (hf.M,) else v) for k, v in res[key].items()}
        rows, fails = compare_solutions(hf, gpu, orc, tol_m, tol_deg, f"serve{key}")
        assert not fails, fails


def test_serving_frames_match_solves_and_oracle(tmp_path):
    """Serving-shaped frames (2/3/4 iterations, hypotheses generated on the
    device around the stream's previous result):
      * with the benchmark's tiles, each served frame equals pilot_solve of
        the same frame from the same prior, bitwise;
      * with tiles whose kernels sum the tap products in FP64 (variant 3),
        the served frames match the oracle on the same bf16-exact inputs at
        the FP32 bar (1 mm / 1e-4 deg, same verdicts)."""
    from paper_2606_31098_amd.pilot import Context, DeviceFrame
    worlds, frames = _serving_inputs()
    say(f"serving {len(frames)} frames of {len(worlds)} sequences with the tile database")
    res = _serve(frames, TILES)
    solo = Context(0, tune_cache=TILES)
    for key in sorted(frames):
        hf, spec = frames[key]
        prior = torch.as_tensor(_prior_of(frames, res, key)[None], device="cuda")
        r = solo.solve([DeviceFrame(hf, dtype="bf16", prior=prior, hyp_offsets=spec.offsets)])[0].numpy()
        for k in ("poses", "cost", "iterations", "status"):
            assert np.array_equal(r[k], res[key][k]), (key, k)
        assert r["best"] == res[key]["best"], key
    solo.close()
    cache = tmp_path / "tiles_v3.txt"
    with open(cache, "w") as fh:
        for hf, _ in frames.values():
            for L in hf.levels:
                fh.write(f"C{L.C}_d1_N{_floor_log2(L.N)}_M{_floor_log2(hf.M)}_P{_floor_log2(L.H * L.W)}_v3 "
                         f"{8 if L.C >= 128 else 4} 2 0 3\n")
    say("serving again with FP64 tap sums (variant 3)")
    res3 = _serve(frames, str(cache))
    last = [(w.seq, len(w.frames) - 1) for w in worlds]
    _against_oracle(frames, res3, [(0, 0), (1, 2)] + last, POSE_TOL_M, POSE_TOL_DEG)


def test_served_bf16_precision_form_matches_oracle_when_converged():
    """The benchmark's tiles (FP32 tap sums on bf16 maps) on serving-shaped
    frames given enough iterations to converge (8 per level): the bf16 bar
    (1 cm / 0.01 deg, same verdicts) against the oracle on the same inputs.
    With the workload's 2/3/4 iterations a hypothesis is still moving by
    metres per step when it stops, so its final pose is no fixed point to
    compare at that bar; the previous test covers that schedule."""
    worlds, frames = _serving_inputs(n_seq=2, iters=(8, 8, 8))
    res = _serve(frames, TILES)
    _against_oracle(frames, res, [(0, 0), (0, 2), (1, 1)], BF16_TOL_M, BF16_TOL_DEG)


def _pruning_frame(seed, M, keep, iters):
    f = S.make_frame(2, 0, N=500, M=M, level_shapes=((60, 80, 32), (120, 160, 64)), iters=iters,
                     dsm_side=128, seed=seed)
    f.keep_top, f.prune_level = keep, 0
    return f


def test_serving_pruning_frames_reuse_freed_ranges():
    """A finished frame's slot stays free while a later frame, admitted into
    another slot, takes over its hypothesis range.  The freed slot's pruning
    descriptor must not rank or prune the newcomer's hypotheses: every result
    equals its frame's pilot_solve, bitwise."""
    from paper_2606_31098_amd.pilot import Context, DeviceFrame, DeviceResult
    fa = S.make_frame(2, 0, N=400, M=16, level_shapes=((60, 80, 32), (120, 160, 64)), iters=(8, 8),
                      dsm_side=128, seed=71)                          # long, no pruning: slot 0
    fb = _pruning_frame(72, 32, 4, (1, 1))                            # short, pruning: slot 1
    fc = S.make_frame(2, 0, N=400, M=8, level_shapes=((60, 80, 32), (120, 160, 64)), iters=(8, 8),
                      dsm_side=128, seed=73)                          # slot 2
    fd = _pruning_frame(74, 40, 10, (4, 4))                           # slot 0 again, over b's old range
    dfs = [DeviceFrame(f) for f in (fa, fb, fc, fd)]
    solo = Context(0)
    ref = [solo.solve([d])[0].numpy() for d in dfs]
    ctx = Context(0, max_slots=3)
    res = [DeviceResult(d.M) for d in dfs]
    slots = {i: ctx.admit(dfs[i], res[i]) for i in range(3)}
    assert slots == {0: 0, 1: 1, 2: 2}, slots
    done, d_slot, steps = set(), None, 0
    say("serving: pruning frames reusing a freed hypothesis range")
    while len(done) < 4:
        ctx.step()
        ctx.sync()
        for i, s in list(slots.items()):
            if ctx.poll(s):
                done.add(i)
                del slots[i]
        if d_slot is None and {0, 1} <= done:
            d_slot = ctx.admit(dfs[3], res[3])
            assert d_slot == 0                               # slot 1 is free and stays free
            slots[3] = d_slot
        steps += 1
        assert steps < 200, "serving did not drain"
    torch.cuda.synchronize()
    for i in range(4):
        got = res[i].numpy()
        for key in ("poses", "cost", "iterations", "status"):
            assert np.array_equal(got[key], ref[i][key]), (i, key)
        assert got["best"] == ref[i]["best"], i
    assert int(np.sum(ref[3]["status"] == oracle.PRUNED)) > 0
