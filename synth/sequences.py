"""Simulated UAV video streams for the serving workload.

16 sequences (by default) fly smooth random trajectories at 100-300 m
altitude with the camera pitched 30-70 deg down; frames arrive as a Poisson
process at 30 Hz per sequence.  Each frame carries a DSM crop of 128-512
samples per side around its view, N = side^2 / 32 lifted anchors, 64-512
hypotheses, a 3-level descriptor pyramid (120x160x32 / 240x320x64 /
480x640x128, bf16) and 2/3/4 LM iterations coarse to fine.

Host-side data (poses, anchors, their ground-truth projections, gravity and
laser-range readings, hypothesis offsets) are drawn before the run from
seeded PCG64 streams.  The descriptor pyramids stand in for the feature
network's output: a ring of them is drawn once on the device with torch
(same recipe as frames.make_field: Gaussian noise, 8 px Gaussian blur with
reflected borders, per-pixel L2 normalisation); frame k uses ring entry
k mod R, and its reference descriptors are bilinear samples of that entry at
the anchors' ground-truth projections plus N(0, 0.05^2) noise, drawn on the
device when the frame arrives.  Nothing here solves anything.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import frames as S

LEVELS = ((120, 160, 32), (240, 320, 64), (480, 640, 128))
ITERS = (2, 3, 4)
RATE_HZ = 30.0


@dataclass
class FrameSpec:
    seq: int
    index: int
    t_arrival: float
    gt_pose: np.ndarray
    P: np.ndarray                 # (N, 3) float32 anchors
    uv: List[np.ndarray]          # per level (N, 2) float64 ground-truth projections
    crop: tuple                   # (i0, j0, side) window of the sequence DSM
    g_imu: np.ndarray
    d_range: float
    offsets: np.ndarray           # (M, 3) dx, dy, dyaw
    init_pose: Optional[np.ndarray] = None   # prior of a sequence's first frame
    noise_seed: int = 0


@dataclass
class SequenceWorld:
    seq: int
    dsm: S.Dsm
    frames: List[FrameSpec] = field(default_factory=list)


def _smooth(rng, t, amp, periods=(20.0, 45.0)):
    """Sum of two slow sinusoids with random phases (amplitude amp)."""
    ph = rng.uniform(0, 2 * math.pi, size=2)
    return amp * 0.5 * (np.sin(2 * math.pi * t / periods[0] + ph[0]) + np.sin(2 * math.pi * t / periods[1] + ph[1]))


def _range_vectorised(dsm: S.Dsm, C: np.ndarray, d: np.ndarray, s_max: float = 2500.0) -> float:
    """Distance along unit d from C to the first DSM crossing: 0.05 m samples
    then bisection to 1e-9 m."""
    s = np.arange(0.0, s_max, 0.05)
    p = C[None, :] + s[:, None] * d[None, :]
    f = p[:, 2] - dsm.height(p[:, 0], p[:, 1])
    hit = np.flatnonzero(f <= 0)
    if hit.size == 0:
        raise ValueError("range ray misses the DSM")
    k = hit[0]
    lo, hi = s[k - 1], s[k]
    while hi - lo > 1e-9:
        mid = 0.5 * (lo + hi)
        pm = C + mid * d
        if pm[2] - dsm.height(pm[0:1], pm[1:2])[0] > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def make_world(seq: int, duration: float, rate_hz: float = RATE_HZ, seed_base: int = S.seed_for(5, 0),
               m_choices=(64, 128, 256, 512)) -> SequenceWorld:
    """One sequence: a 2048x2048 DSM (1 km at 0.5 m), a trajectory and its
    frames' host-side data."""
    ss = np.random.SeedSequence(seed_base + 97 * seq)
    r_dsm, r_traj, r_arr, r_fr = [np.random.Generator(np.random.PCG64(x)) for x in ss.spawn(4)]
    dsm = S.make_dsm(r_dsm, 2048)
    # arrivals: Poisson process
    ts, t = [], r_arr.exponential(1.0 / rate_hz)
    while t < duration:
        ts.append(t)
        t += r_arr.exponential(1.0 / rate_hz)
    ts = np.array(ts)
    # ground footprint of the optical axis moves at ~10 m/s inside +-300 m
    heading0 = r_traj.uniform(0, 2 * math.pi)
    start = r_traj.uniform(-150, 150, size=2)
    turn = _smooth(r_traj, ts, 0.6)                     # heading wobble (rad)
    alt = 200.0 + _smooth(r_traj, ts, 100.0)            # 100..300 m
    pitch = np.radians(50.0 + _smooth(r_traj, ts, 20.0))   # 30..70 deg down
    roll = np.radians(_smooth(r_traj, ts, 3.0))
    world = SequenceWorld(seq=seq, dsm=dsm)
    fp = start.copy()
    prev_t = 0.0
    for k, t in enumerate(ts):
        hd = heading0 + turn[k]
        fp = fp + 10.0 * (t - prev_t) * np.array([math.sin(hd), math.cos(hd)])
        fp = np.clip(fp, -300.0, 300.0)
        prev_t = t
        yaw = -hd                                       # camera looks along the heading
        R_wc = S.camera_to_world_rotation(yaw, pitch[k], roll[k])
        axis = R_wc @ np.array([0.0, 0.0, 1.0])
        target = np.array([fp[0], fp[1], float(dsm.height(fp[0:1], fp[1:2])[0])])
        C = target - (alt[k] / -axis[2]) * axis
        gt = S.pose_from_center(R_wc, C)
        side = int(r_fr.integers(128, 513))
        N = side * side // 32
        M = int(r_fr.choice(m_choices))
        cj = int(round((fp[0] - dsm.x0) / dsm.gsd)) - side // 2
        ci = int(round((fp[1] - dsm.y0) / dsm.gsd)) - side // 2
        cj = int(np.clip(cj, 0, 2048 - side))
        ci = int(np.clip(ci, 0, 2048 - side))
        # anchors: random crop samples in front of and inside every level
        chosen, have = [], 0
        R = gt[:9].reshape(3, 3)
        tries = 0
        while have < N and tries < 20:
            ii = r_fr.integers(0, side, size=3 * (N - have))
            jj = r_fr.integers(0, side, size=3 * (N - have))
            P = np.stack([dsm.x0 + (cj + jj) * dsm.gsd, dsm.y0 + (ci + ii) * dsm.gsd,
                          dsm.heights[ci + ii, cj + jj].astype(np.float64)], 1).astype(np.float32).astype(np.float64)
            X = P @ R.T + gt[9:]
            ok = X[:, 2] > 1.0
            for (H, W, _) in LEVELS:
                fx, fy, cx, cy = S.level_intrinsics(H, W)
                u = fx * X[:, 0] / X[:, 2] + cx
                v = fy * X[:, 1] / X[:, 2] + cy
                ok &= (u >= 1) & (u <= W - 2) & (v >= 1) & (v <= H - 2)
            chosen.append(P[ok][:N - have])
            have += len(chosen[-1])
            tries += 1
        if have < N:
            raise ValueError(f"sequence {seq} frame {k}: only {have} of {N} anchors in view")
        P = np.concatenate(chosen)[:N]
        X = P @ R.T + gt[9:]
        uv = []
        for (H, W, _) in LEVELS:
            fx, fy, cx, cy = S.level_intrinsics(H, W)
            uv.append(np.stack([fx * X[:, 0] / X[:, 2] + cx, fy * X[:, 1] / X[:, 2] + cy], 1))
        g_imu = S.gravity_in_camera(pitch[k] + math.radians(r_fr.normal(0, S.GRAVITY_NOISE_DEG)),
                                    roll[k] + math.radians(r_fr.normal(0, S.GRAVITY_NOISE_DEG)))
        d = _range_vectorised(dsm, C, axis) + r_fr.normal(0, S.RANGE_NOISE_M)
        offs = np.stack([r_fr.uniform(-S.HYP_TRANS_M, S.HYP_TRANS_M, M),
                         r_fr.uniform(-S.HYP_TRANS_M, S.HYP_TRANS_M, M),
                         np.radians(r_fr.uniform(-S.HYP_YAW_DEG, S.HYP_YAW_DEG, M))], 1)
        offs[0] = 0.0                                   # hypothesis 0 is the prior itself
        spec = FrameSpec(seq=seq, index=k, t_arrival=float(t), gt_pose=gt, P=P.astype(np.float32), uv=uv,
                         crop=(ci, cj, side), g_imu=g_imu, d_range=float(d), offsets=offs,
                         noise_seed=int(seed_base + 7919 * seq + k))
        if k == 0:
            spec.init_pose = S.perturb_pose(r_fr, gt, S.INIT_TRANS_M, S.INIT_ROT_DEG)
        world.frames.append(spec)
    return world


# ---------------------------------------------------------------------- device side
def make_field_torch(H, W, C, sigma, gen, device):
    """Device version of frames.make_field (bf16 result)."""
    import torch
    import torch.nn.functional as Fn
    x = torch.randn((1, C, H, W), generator=gen, device=device, dtype=torch.float32)
    r = int(math.ceil(4 * sigma))
    k = torch.exp(-0.5 * (torch.arange(-r, r + 1, device=device, dtype=torch.float32) / sigma) ** 2)
    k = k / k.sum()
    x = Fn.pad(x, (r, r, 0, 0), mode="reflect")
    x = Fn.conv2d(x, k.view(1, 1, 1, -1).expand(C, 1, 1, -1).contiguous(), groups=C)
    x = Fn.pad(x, (0, 0, r, r), mode="reflect")
    x = Fn.conv2d(x, k.view(1, 1, -1, 1).expand(C, 1, -1, 1).contiguous(), groups=C)
    x = x[0].permute(1, 2, 0).contiguous()
    x = x / torch.linalg.vector_norm(x, dim=2, keepdim=True)
    return x.to(torch.bfloat16).contiguous()


def pyramid_ring(R: int, device="cuda", seed: int = S.seed_for(5, 999)):
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return [[make_field_torch(H, W, C, S.FEATURE_SIGMA_PX, gen, device) for (H, W, C) in LEVELS] for _ in range(R)]


def sample_reference(feat, uv, noise_seed, device="cuda"):
    """Bilinear samples of a bf16 (H, W, C) map at (N, 2) positions plus
    N(0, 0.05^2) noise, rounded to bf16 (device, torch)."""
    import torch
    H, W, C = feat.shape
    u = torch.as_tensor(uv[:, 0], device=device)
    v = torch.as_tensor(uv[:, 1], device=device)
    x0 = torch.clamp(torch.floor(u), max=W - 2).long()
    y0 = torch.clamp(torch.floor(v), max=H - 2).long()
    a = (u - x0).float()[:, None]
    b = (v - y0).float()[:, None]
    f = feat.float()
    val = ((1 - a) * (1 - b) * f[y0, x0] + a * (1 - b) * f[y0, x0 + 1]
           + (1 - a) * b * f[y0 + 1, x0] + a * b * f[y0 + 1, x0 + 1])
    g = torch.Generator(device=device)
    g.manual_seed(noise_seed)
    val = val + S.FEATURE_NOISE * torch.randn(val.shape, generator=g, device=device)
    return val.to(torch.bfloat16).contiguous()
