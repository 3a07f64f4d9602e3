"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (the committed tile database): the GPU solves the whole
workload, the oracle solves a sample of hypotheses one by one at full N."""
import os

import numpy as np
import pytest
import torch

import oracle
from synth import frames as S
from tests.gpu_common import BF16_TOL_DEG, BF16_TOL_M, POSE_TOL_DEG, POSE_TOL_M, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TILES = os.path.join(ROOT, "paper_2606_31098_amd", "tiles_gfx950.txt")


def _solve(frames, dtype):
    from paper_2606_31098_amd.pilot import Context, DeviceFrame
    ctx = Context(0, tune_cache=TILES)
    dfs = [DeviceFrame(f, dtype=dtype) for f in frames]
    res = ctx.solve(dfs)
    torch.cuda.synchronize()
    out = [r.numpy() for r in res]
    ctx.close()
    return out


def _check_sample(frame, gpu, hyps, tol_m, tol_deg, orc=None):
    """Verdicts and poses of hypotheses `hyps` against the oracle (which
    solves them one by one at full N unless its result is given)."""
    if orc is None:
        orc = oracle.solve(frame, hyps=hyps, threads=0)
    te_g, re_g = S.pose_errors(gpu["poses"][hyps], frame.gt_pose)
    te_o, re_o = S.pose_errors(orc["poses"], frame.gt_pose)
    vg, vo = (te_g <= 1.0) & (re_g <= 1.0), (te_o <= 1.0) & (re_o <= 1.0)
    assert np.array_equal(vg, vo), (hyps[vg != vo], vg.sum(), vo.sum())
    worst = (0.0, 0.0)
    for k, m in enumerate(hyps):
        if vo[k]:
            dt, dr = S.pose_errors(gpu["poses"][m], orc["poses"][k])
            worst = (max(worst[0], dt[0]), max(worst[1], dr[0]))
            assert dt[0] <= tol_m and dr[0] <= tol_deg, (m, dt, dr)
    say(f"{len(hyps)} hypotheses, {int(vo.sum())} converged in both: worst {worst[0]:.2e} m / {worst[1]:.2e} deg")
    return orc


def test_config2_full_size_f32_and_bf16():
    """Every one of the 256 hypotheses of the full-size pyramid frame."""
    f = S.make_frame(2, 0)                   # 3 levels up to 480x640x128, N = 8192, M = 256
    hyps = np.arange(f.M)
    say("config 2 f32")
    gpu = _solve([f], "f32")[0]
    orc = _check_sample(f, gpu, hyps, POSE_TOL_M, POSE_TOL_DEG)
    say("config 2 bf16 (precision form) against the oracle on the f32 inputs")
    gpub = _solve([f], "bf16")[0]
    _check_sample(f, gpub, hyps, BF16_TOL_M, BF16_TOL_DEG, orc=orc)


def test_config3_full_size_bf16():
    f = S.make_frame(3, 0)                   # N = 16384, M = 1024, bf16 maps
    hyps = np.arange(0, f.M, 16)             # 64 hypotheses spread over the tiles
    say("config 3 bf16")
    gpu = _solve([f], "bf16")[0]
    _check_sample(f, gpu, hyps, BF16_TOL_M, BF16_TOL_DEG)


def test_config4_batch_frames_full_size_bf16():
    frames = S.make_batch(64, field_pool=4)  # 64 uneven frames in one solve
    say("config 4 bf16, 64 frames")
    out = _solve(frames, "bf16")
    for i in (0, 31, 63):
        f = frames[i]
        hyps = np.unique(np.linspace(0, f.M - 1, 8).astype(int))
        _check_sample(f, out[i], hyps, BF16_TOL_M, BF16_TOL_DEG)
