"""Seeded synthetic frames shaped like the paper's registration workloads.

The paper evaluates on SynthCity-6, UAVScenes and UAVD4L-2yr, none of which
is available here; these generators stand in for them.  Nothing in this module
solves anything: it builds a synthetic scene (DSM crop, a ground-truth oblique
camera, a query feature pyramid) and the measurements a solver receives
(lifted 3D anchors with reference descriptors, gravity and laser-range
readings, initial pose hypotheses).  To make the measurements self-consistent
it contains its own scene-synthesis camera: ground-truth pinhole projection,
bilinear resampling of the synthetic feature field and a ray march against the
DSM.  Neither the FP64 oracle nor the GPU library imports this module; only
the arrays it returns are handed to both.

Conventions shared with every consumer (they describe the data, not the
solver):
  * world frame: local ENU in metres, z up, gravity direction (0, 0, -1);
  * camera frame: x right, y down, z forward (pixel centres at integers);
  * a pose is world->camera, 12 float64: R row-major (9) then t (3),
    X_cam = R @ X_world + t;
  * feature maps are channels-last (H, W, C), descriptors L2-normalised per
    pixel before the reference features are sampled (network description,
    supplement "Network Architecture");
  * the DSM crop is (Hd, Wd) heights, sample (i, j) sits at world
    (x0 + j*gsd, y0 + i*gsd).

Every random draw comes from numpy's PCG64 seeded with
31098 + 1000*config + frame; each component draws from its own spawned
child stream so that changing one size leaves the other components intact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.fft

GSD = 0.5                      # metres per DSM sample
FEATURE_SIGMA_PX = 8.0         # smoothness of the synthetic descriptor field
FEATURE_NOISE = 0.05           # per-channel reference-descriptor noise
GRAVITY_NOISE_DEG = 0.5        # roll/pitch noise of the IMU reading
RANGE_NOISE_M = 0.5            # laser range noise
INIT_TRANS_M = 5.0             # initial-prior translation error
INIT_ROT_DEG = 3.0             # initial-prior rotation error
HYP_TRANS_M = 20.0             # hypotheses: x, y offsets in [-20, 20] m
HYP_YAW_DEG = 10.0             # hypotheses: yaw offsets in [-10, 10] deg

LOSS_CAUCHY, LOSS_HUBER, LOSS_L2 = 0, 1, 2


def seed_for(config: int, frame: int) -> int:
    return 31098 + 1000 * config + frame


# --------------------------------------------------------------------------
# small rotation helpers (scene synthesis only)
# --------------------------------------------------------------------------
def _rz(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rx(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


# camera (x right, y down, z forward) -> world (x east, y north, z up) at
# zero yaw/pitch/roll: the camera looks north along the horizon.
_B = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, -1.0, 0.0]])


def camera_to_world_rotation(yaw: float, pitch_down: float, roll: float) -> np.ndarray:
    """R_wc = Rz(yaw) B Rx(-pitch_down) Rz(roll) (radians)."""
    return _rz(yaw) @ _B @ _rx(-pitch_down) @ _rz(roll)


def gravity_in_camera(pitch_down: float, roll: float) -> np.ndarray:
    """Unit gravity direction seen in the camera frame for R_wc above.

    Written from the angles (not from a rotation matrix) so that it is an
    independent statement of what an IMU reports.
    """
    cp = math.cos(pitch_down)
    return np.array([cp * math.sin(roll), cp * math.cos(roll), math.sin(pitch_down)])


def _axis_angle(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation matrix from a unit axis and an angle (scene synthesis)."""
    k = axis / np.linalg.norm(axis)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def pose_from_center(R_wc: np.ndarray, C: np.ndarray) -> np.ndarray:
    """World->camera 12-vector from a camera-to-world rotation and centre."""
    R = R_wc.T
    t = -R @ C
    return np.concatenate([R.reshape(-1), t])


def center_of(pose: np.ndarray) -> np.ndarray:
    R = pose[:9].reshape(3, 3)
    return -R.T @ pose[9:]


def _uniform_unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# DSM crop
# --------------------------------------------------------------------------
@dataclass
class Dsm:
    heights: np.ndarray          # (Hd, Wd) float32
    x0: float
    y0: float
    gsd: float

    def height(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        """Bilinear height with clamp-to-edge, float64 arithmetic on the
        float32 raster (the same surface a solver sees)."""
        Hd, Wd = self.heights.shape
        D = self.heights
        fj = np.clip((np.asarray(x, np.float64) - self.x0) / self.gsd, 0.0, Wd - 1.0)
        fi = np.clip((np.asarray(y, np.float64) - self.y0) / self.gsd, 0.0, Hd - 1.0)
        j0 = np.minimum(np.floor(fj).astype(np.int64), Wd - 2)
        i0 = np.minimum(np.floor(fi).astype(np.int64), Hd - 2)
        a = fj - j0
        b = fi - i0
        d00, d01 = D[i0, j0].astype(np.float64), D[i0, j0 + 1].astype(np.float64)
        d10, d11 = D[i0 + 1, j0].astype(np.float64), D[i0 + 1, j0 + 1].astype(np.float64)
        top = d00 * (1.0 - a) + d01 * a
        bot = d10 * (1.0 - a) + d11 * a
        return top * (1.0 - b) + bot * b


def make_dsm(rng: np.random.Generator, side: int, gsd: float = GSD) -> Dsm:
    """Sum of 8 isotropic Gaussians normalised to [0, 50] m plus 4 box
    'buildings' 10-40 m tall; crop centred on the world origin."""
    ext = (side - 1) * gsd
    x0 = y0 = -0.5 * ext
    jj, ii = np.meshgrid(np.arange(side), np.arange(side))
    X = x0 + jj * gsd
    Y = y0 + ii * gsd
    h = np.zeros((side, side))
    for _ in range(8):
        cx, cy = rng.uniform(-0.75 * ext, 0.75 * ext, size=2)
        sig = rng.uniform(0.1, 0.4) * ext
        amp = rng.uniform(0.5, 1.0)
        h += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig * sig))
    h = (h - h.min()) / max(h.max() - h.min(), 1e-12) * 50.0
    for _ in range(4):
        w, l = rng.uniform(0.1, 0.25, size=2) * side
        ci, cj = rng.uniform(0, side, size=2)
        i_lo, i_hi = int(max(0, ci - l / 2)), int(min(side, ci + l / 2))
        j_lo, j_hi = int(max(0, cj - w / 2)), int(min(side, cj + w / 2))
        h[i_lo:i_hi, j_lo:j_hi] += rng.uniform(10.0, 40.0)
    return Dsm(h.astype(np.float32), float(x0), float(y0), float(gsd))


# --------------------------------------------------------------------------
# feature field
# --------------------------------------------------------------------------
def make_field(rng: np.random.Generator, H: int, W: int, C: int,
               sigma: float = FEATURE_SIGMA_PX) -> np.ndarray:
    """Smooth Gaussian random field, per-pixel L2-normalised, (H, W, C) f32.

    i.i.d. N(0,1) per channel, Gaussian blur of std `sigma` pixels with
    reflected borders (FFT convolution on a 4-sigma reflect pad)."""
    pad = int(math.ceil(4 * sigma))
    noise = rng.standard_normal((H, W, C), dtype=np.float32)
    x = np.pad(noise, ((pad, pad), (pad, pad), (0, 0)), mode="reflect")
    Hp, Wp = x.shape[:2]
    fy = np.fft.fftfreq(Hp)[:, None]
    fx = np.fft.rfftfreq(Wp)[None, :]
    tf = np.exp(-2.0 * (math.pi * sigma) ** 2 * (fy ** 2 + fx ** 2)).astype(np.float32)
    X = scipy.fft.rfft2(x, axes=(0, 1), workers=-1)
    X *= tf[:, :, None]
    y = scipy.fft.irfft2(X, s=(Hp, Wp), axes=(0, 1), workers=-1)[pad:pad + H, pad:pad + W]
    y = y / np.linalg.norm(y, axis=2, keepdims=True)
    return np.ascontiguousarray(y, dtype=np.float32)


def sample_field(F: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Bilinear samples (float64) of a channels-last field at (u, v)."""
    H, W, _ = F.shape
    F = F.astype(np.float64)
    x0 = np.minimum(np.floor(u).astype(np.int64), W - 2)
    y0 = np.minimum(np.floor(v).astype(np.int64), H - 2)
    a = (u - x0)[:, None]
    b = (v - y0)[:, None]
    return ((1 - a) * (1 - b) * F[y0, x0] + a * (1 - b) * F[y0, x0 + 1]
            + (1 - a) * b * F[y0 + 1, x0] + a * b * F[y0 + 1, x0 + 1])


# --------------------------------------------------------------------------
# frames
# --------------------------------------------------------------------------
def level_intrinsics(H: int, W: int, H0: int = 120, f0: float = 140.0):
    """Pinhole intrinsics of an (H, W) level of a pyramid whose (120, 160)
    level has f = 140 px; principal point at the image centre."""
    s = H / H0
    return (f0 * s, f0 * s, (W - 1) / 2.0, (H - 1) / 2.0)


def default_losses(C: int):
    """Photo loss per level (Cauchy, scale 0.1*C/32 ~ 1.25x the descriptor
    noise floor C*0.05^2)."""
    return (LOSS_CAUCHY, 0.1 * C / 32.0)


GRAVITY_LOSS = (LOSS_HUBER, (3.0 * math.radians(GRAVITY_NOISE_DEG)) ** 2)
RANGE_LOSS = (LOSS_HUBER, (3.0 * RANGE_NOISE_M) ** 2)
LAMBDA_IMU = FEATURE_NOISE ** 2 / math.radians(GRAVITY_NOISE_DEG) ** 2
LAMBDA_RANGE = FEATURE_NOISE ** 2 / RANGE_NOISE_M ** 2
# adaptive prior scales: a prior's gradient is capped at ALPHA_RATIO times
# the visual gradient, and residuals beyond 5 sigma are gated down
ALPHA_RATIO = 1.0
GRAVITY_GATE = 5.0 * math.radians(GRAVITY_NOISE_DEG)
RANGE_GATE = 5.0 * RANGE_NOISE_M

LM_DEFAULTS = dict(tau=1e-6, up=10.0, down=10.0, lambda_min_rel=1e-12,
                   lambda_max_rel=1e8, step_tol_t=1e-5, step_tol_r=1e-7,
                   z_min=0.1, min_valid=8, cost_tol=1e-6)


@dataclass
class Level:
    H: int
    W: int
    C: int
    feat: np.ndarray            # (H, W, C) float32
    K: tuple                    # (fx, fy, cx, cy)
    x: np.ndarray               # (N,) float32
    y: np.ndarray
    z: np.ndarray
    ref: np.ndarray             # (N, C) float32
    iters: int
    loss: tuple                 # (kind, scale)
    ref_w: Optional[np.ndarray] = None   # (N,) float32
    qconf: Optional[np.ndarray] = None   # (H, W) float32

    @property
    def N(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Frame:
    levels: List[Level]                  # coarse -> fine
    poses: np.ndarray                    # (M, 12) float64 world->camera
    dsm: Dsm
    g_imu: np.ndarray                    # (3,)
    d_range: float
    pc: tuple                            # range pixel on the finest level
    use_gravity: int = 1
    use_range: int = 1
    g_world: tuple = (0.0, 0.0, -1.0)
    lambda_imu: float = LAMBDA_IMU
    lambda_range: float = LAMBDA_RANGE
    gravity_loss: tuple = GRAVITY_LOSS
    range_loss: tuple = RANGE_LOSS
    lm: dict = field(default_factory=lambda: dict(LM_DEFAULTS))
    gt_pose: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)
    keep_top: int = 0                   # top-K pruning after prune_level (0 = none)
    prune_level: int = 0
    adaptive_priors: int = 0            # adaptive prior scales with residual gates
    alpha_ratio: float = ALPHA_RATIO
    gravity_gate: float = GRAVITY_GATE
    range_gate: float = RANGE_GATE

    @property
    def M(self) -> int:
        return int(self.poses.shape[0])


def _gt_camera(rng, altitude=150.0, pitch_deg=45.0, roll_max_deg=3.0, target=(0.0, 0.0)):
    yaw = rng.uniform(0.0, 2.0 * math.pi)
    roll = math.radians(rng.uniform(-roll_max_deg, roll_max_deg))
    pitch = math.radians(pitch_deg)
    R_wc = camera_to_world_rotation(yaw, pitch, roll)
    axis = R_wc @ np.array([0.0, 0.0, 1.0])           # optical axis in world
    s = altitude / -axis[2]
    C = np.array([target[0], target[1], 0.0]) - s * axis
    return R_wc, C, pitch, roll


def _project(pose: np.ndarray, K, P: np.ndarray):
    R = pose[:9].reshape(3, 3)
    Xc = P @ R.T + pose[9:]
    fx, fy, cx, cy = K
    return fx * Xc[:, 0] / Xc[:, 2] + cx, fy * Xc[:, 1] / Xc[:, 2] + cy, Xc[:, 2]


def _range_along_axis(dsm: Dsm, C: np.ndarray, d: np.ndarray, s_max: float = 2000.0) -> float:
    """Distance from C along unit d to the first crossing of the bilinear
    DSM: 0.05 m march, then bisection to 1e-9 m."""
    step = 0.05
    s0 = 0.0
    f0 = C[2] - dsm.height(C[0:1], C[1:2])[0]
    if f0 <= 0:
        raise ValueError("camera below the surface")
    s = step
    while s < s_max:
        p = C + s * d
        f = p[2] - dsm.height(p[0:1], p[1:2])[0]
        if f <= 0:
            lo, hi = s0, s
            while hi - lo > 1e-9:
                mid = 0.5 * (lo + hi)
                pm = C + mid * d
                if pm[2] - dsm.height(pm[0:1], pm[1:2])[0] > 0:
                    lo = mid
                else:
                    hi = mid
            return 0.5 * (lo + hi)
        s0 = s
        s += step
    raise ValueError("range ray does not hit the DSM")


def perturb_pose(rng, pose: np.ndarray, trans_m: float, rot_deg: float) -> np.ndarray:
    """C += trans_m in a uniform direction; R_wc <- R_wc Exp(rot about a
    uniform axis)."""
    R_wc = pose[:9].reshape(3, 3).T
    C = center_of(pose) + trans_m * _uniform_unit(rng)
    R_wc = R_wc @ _axis_angle(_uniform_unit(rng), math.radians(rot_deg))
    return pose_from_center(R_wc, C)


def hypothesis(pose: np.ndarray, dx: float, dy: float, dyaw: float) -> np.ndarray:
    """Shift a pose by (dx, dy) metres and rotate it by dyaw about the world
    z axis through its camera centre; height, roll and pitch unchanged."""
    R_wc = pose[:9].reshape(3, 3).T
    C = center_of(pose) + np.array([dx, dy, 0.0])
    return pose_from_center(_rz(dyaw) @ R_wc, C)


def random_hypotheses(rng, prior: np.ndarray, M: int,
                      trans_m: float = HYP_TRANS_M, yaw_deg: float = HYP_YAW_DEG) -> np.ndarray:
    """m = 0 is the prior itself; m >= 1 draw dx, dy ~ U[-trans, trans] m
    and dyaw ~ U[-yaw, yaw] deg around it."""
    out = np.empty((M, 12))
    out[0] = prior
    for m in range(1, M):
        dx, dy = rng.uniform(-trans_m, trans_m, size=2)
        dpsi = math.radians(rng.uniform(-yaw_deg, yaw_deg))
        out[m] = hypothesis(prior, dx, dy, dpsi)
    return out


def paper_grid_offsets():
    """(dx, dy, dyaw) of the paper's hypothesis grid: x, y in -10..10 m step
    2 m, yaw offsets +-1, 3, 5, 7, 9 deg (supplement, Multi-Hypothesis
    Refinement): 11 * 11 * 10 = 1210 entries."""
    xs = np.arange(-10.0, 10.0 + 1e-9, 2.0)
    yaws = [math.radians(s * a) for a in (1, 3, 5, 7, 9) for s in (1, -1)]
    return [(dx, dy, dpsi) for dx in xs for dy in xs for dpsi in yaws]


def grid_hypotheses(prior: np.ndarray) -> np.ndarray:
    return np.stack([hypothesis(prior, dx, dy, dp) for dx, dy, dp in paper_grid_offsets()])


def make_frame(config: int = 2, frame: int = 0, *, noise: bool = True,
               N: Optional[int] = None, M: Optional[int] = None,
               level_shapes=None, iters=None, dsm_side: Optional[int] = None,
               seed: Optional[int] = None, feature_sigma: float = FEATURE_SIGMA_PX,
               altitude: float = 150.0, pitch_deg: float = 45.0,
               field_cache: Optional[dict] = None, field_key: int = 0) -> Frame:
    """One synthetic frame.

    config 1: 64x64 DSM, N=1024, M=1, one 120x160x32 level, 20 iterations.
    config 2: 256x256 DSM, N=8192, M=256, levels 120x160x32 / 240x320x64 /
              480x640x128, 15 iterations per level.
    config 3: as config 2 with N=16384 and M=1024 (the caller rounds the maps
              and reference descriptors to bf16).
    Keyword arguments override the sizes (used for small test cases).
    field_cache: optional dict shared across frames; the descriptor field of
    an (H, W, C) level is then drawn once per (H, W, C, field_key) and reused
    (each frame still gets its own anchors, poses and reference samples).
    """
    presets = {
        1: dict(dsm_side=64, N=1024, M=1, levels=[(120, 160, 32)], iters=[20]),
        2: dict(dsm_side=256, N=8192, M=256,
                levels=[(120, 160, 32), (240, 320, 64), (480, 640, 128)], iters=[15, 15, 15]),
        3: dict(dsm_side=256, N=16384, M=1024,
                levels=[(120, 160, 32), (240, 320, 64), (480, 640, 128)], iters=[15, 15, 15]),
    }
    p = dict(presets.get(config, presets[2]))
    if N is not None:
        p["N"] = N
    if M is not None:
        p["M"] = M
    if level_shapes is not None:
        p["levels"] = list(level_shapes)
    if iters is not None:
        p["iters"] = list(iters)
    if dsm_side is not None:
        p["dsm_side"] = dsm_side
    if len(p["iters"]) != len(p["levels"]):
        p["iters"] = [p["iters"][0]] * len(p["levels"])

    ss = np.random.SeedSequence(seed if seed is not None else seed_for(config, frame))
    (r_dsm, r_cam, r_pts, r_init, r_grav, r_rng, r_hyp, r_ref,
     *r_fields) = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(8 + len(p["levels"]))]

    dsm = make_dsm(r_dsm, p["dsm_side"])
    R_wc, Cgt, pitch, roll = _gt_camera(r_cam, altitude=altitude, pitch_deg=pitch_deg)
    gt = pose_from_center(R_wc, Cgt)

    # candidate anchors: every DSM sample in front of and inside every level
    Hd, Wd = dsm.heights.shape
    jj, ii = np.meshgrid(np.arange(Wd), np.arange(Hd))
    P = np.stack([(dsm.x0 + jj * dsm.gsd).ravel(), (dsm.y0 + ii * dsm.gsd).ravel(),
                  dsm.heights.astype(np.float64).ravel()], axis=1)
    P = P.astype(np.float32).astype(np.float64)
    ok = np.ones(P.shape[0], bool)
    for (H, W, C) in p["levels"]:
        u, v, Z = _project(gt, level_intrinsics(H, W), P)
        ok &= (Z > 1.0) & (u >= 1.0) & (u <= W - 2.0) & (v >= 1.0) & (v <= H - 2.0)
    cand = np.flatnonzero(ok)
    if cand.size < p["N"]:
        raise ValueError(f"only {cand.size} anchors visible, {p['N']} requested")
    idx = np.sort(r_pts.choice(cand, size=p["N"], replace=False))   # DSM row-major order
    P = P[idx]

    levels = []
    for li, (H, W, C) in enumerate(p["levels"]):
        K = level_intrinsics(H, W)
        if field_cache is not None:
            fk = (H, W, C, field_key)
            if fk not in field_cache:
                field_cache[fk] = make_field(np.random.default_rng(seed_for(9, H * 7 + W * 13 + C * 17 + 1009 * field_key)), H, W, C,
                                             feature_sigma)
            F = field_cache[fk]
        else:
            F = make_field(r_fields[li], H, W, C, feature_sigma)
        u, v, _ = _project(gt, K, P)
        ref = sample_field(F, u, v)
        if noise:
            ref = ref + r_ref.normal(0.0, FEATURE_NOISE, size=ref.shape)
        levels.append(Level(H=H, W=W, C=C, feat=F, K=K,
                            x=P[:, 0].astype(np.float32), y=P[:, 1].astype(np.float32),
                            z=P[:, 2].astype(np.float32), ref=ref.astype(np.float32),
                            iters=p["iters"][li], loss=default_losses(C)))

    init = perturb_pose(r_init, gt, INIT_TRANS_M, INIT_ROT_DEG)
    poses = random_hypotheses(r_hyp, init, p["M"])

    if noise:
        g_imu = gravity_in_camera(pitch + math.radians(r_grav.normal(0, GRAVITY_NOISE_DEG)),
                                  roll + math.radians(r_grav.normal(0, GRAVITY_NOISE_DEG)))
    else:
        g_imu = gravity_in_camera(pitch, roll)

    Hf, Wf, _ = p["levels"][-1]
    fxf, fyf, cxf, cyf = level_intrinsics(Hf, Wf)
    pc = (cxf, cyf)
    ray_c = np.array([(pc[0] - cxf) / fxf, (pc[1] - cyf) / fyf, 1.0])
    ray_c /= np.linalg.norm(ray_c)
    d = _range_along_axis(dsm, Cgt, R_wc @ ray_c)
    if noise:
        d += r_rng.normal(0.0, RANGE_NOISE_M)

    return Frame(levels=levels, poses=poses, dsm=dsm, g_imu=g_imu, d_range=float(d), pc=pc,
                 gt_pose=gt, meta=dict(config=config, frame=frame, noise=noise,
                                       pitch=pitch, roll=roll, init_pose=init))


def paper_shaped_frame(frame: int = 0) -> Frame:
    """The paper's own online workload shape (Experiments, Implementation
    Details; supplement, Multi-Hypothesis Refinement): 500 anchors, the
    1210-hypothesis (x, y, yaw) grid around the prior, top 128 kept after the
    coarse level, 2/3/4 iterations coarse to fine, 32-channel descriptors at
    every level (sizes as the default pyramid)."""
    f = make_frame(0, frame, N=500, M=1, level_shapes=((120, 160, 32), (240, 320, 32), (480, 640, 32)),
                   iters=(2, 3, 4), dsm_side=256)
    f.poses = grid_hypotheses(f.meta["init_pose"])
    f.keep_top, f.prune_level = 128, 0
    return f


def batch_config(n: int = 64, seed: int = seed_for(4, 0)):
    """Shapes of the uneven batch: per frame N log-uniform in [2048, 32768],
    M uniform in {32, 64, 128, 256, 512}, finest level one of 240x320,
    360x480, 480x640 (levels at 1/4, 1/2, 1 of it with C = 32, 64, 128),
    15 LM iterations per level."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(math.floor(math.exp(rng.uniform(math.log(2048), math.log(32768)))))
        M = int(rng.choice([32, 64, 128, 256, 512]))
        Hf, Wf = [(240, 320), (360, 480), (480, 640)][int(rng.integers(0, 3))]
        levels = ((Hf // 4, Wf // 4, 32), (Hf // 2, Wf // 2, 64), (Hf, Wf, 128))
        out.append(dict(N=N, M=M, level_shapes=levels, iters=(15, 15, 15)))
    return out


def make_batch(n: int = 64, field_pool: int = 8, progress=None) -> List[Frame]:
    """The uneven batch (see batch_config); descriptor fields come from a pool
    of `field_pool` fields per level shape (frames keep their own anchors,
    poses, DSM and reference samples)."""
    cache: dict = {}
    frames = []
    for i, kw in enumerate(batch_config(n)):
        frames.append(make_frame(4, i, dsm_side=256, field_cache=cache, field_key=i % field_pool, **kw))
        if progress:
            progress(i)
    return frames


# --------------------------------------------------------------------------
# pose error metrics (harness only)
# --------------------------------------------------------------------------
def pose_errors(poses: np.ndarray, ref_pose: np.ndarray):
    """Translation error of the camera centre (m) and rotation error (deg)."""
    poses = np.atleast_2d(poses)
    Cr = center_of(ref_pose)
    Rr = ref_pose[:9].reshape(3, 3)
    te = np.empty(len(poses))
    re = np.empty(len(poses))
    for i, p in enumerate(poses):
        te[i] = np.linalg.norm(center_of(p) - Cr)
        Rd = p[:9].reshape(3, 3) @ Rr.T
        c = np.clip((np.trace(Rd) - 1.0) / 2.0, -1.0, 1.0)
        s = np.linalg.norm([Rd[2, 1] - Rd[1, 2], Rd[0, 2] - Rd[2, 0], Rd[1, 0] - Rd[0, 1]]) / 2.0
        re[i] = math.degrees(math.atan2(s, c))
    return te, re
