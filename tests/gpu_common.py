"""Shared helpers of the GPU parity tests (frames, rounding, comparisons)."""
import copy
import sys

import numpy as np
import torch

from synth import frames as S

POSE_TOL_M = 1e-3          # FP32 path: final pose within 1 mm ...
POSE_TOL_DEG = 1e-4        # ... and 1e-4 degrees of the FP64 oracle
BF16_TOL_M = 1e-2          # BF16 path: 1 cm ...
BF16_TOL_DEG = 1e-2        # ... and 0.01 degrees
NEQ_TOL = 1e-5             # normal equations: relative Frobenius error of [H | g]
VERDICT_M, VERDICT_DEG = 1.0, 1.0   # converged <=> within 1 m and 1 deg of ground truth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16_round(a: np.ndarray) -> np.ndarray:
    """float32 values rounded to bfloat16 (round-to-nearest-even) and back."""
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).to(torch.bfloat16).to(torch.float32).numpy()


def bf16_copy(frame):
    f = copy.deepcopy(frame)
    for L in f.levels:
        L.feat = bf16_round(L.feat)
        L.ref = bf16_round(L.ref)
    return f


def project(L, pose):
    R = pose[:9].reshape(3, 3)
    P = np.stack([L.x, L.y, L.z], 1).astype(np.float64)
    X = P @ R.T + pose[9:]
    return L.K[0] * X[:, 0] / X[:, 2] + L.K[2], L.K[1] * X[:, 1] / X[:, 2] + L.K[3]


def mask_edges(frame, poses, eps=1e-3):
    """ref_w = 0 for anchors whose FP64 projection under any of `poses` lies
    within eps px of a pixel row/column (the bilinear gradient jumps there
    and FP32 may land on the other side)."""
    for L in frame.levels:
        w = np.ones(len(L.x), np.float32) if L.ref_w is None else L.ref_w.copy()
        for p in np.atleast_2d(poses):
            u, v = project(L, p)
            w[(np.abs(u - np.round(u)) < eps) | (np.abs(v - np.round(v)) < eps)] = 0.0
        L.ref_w = w
    return frame


def border_count(L, pose, eps=1e-3):
    u, v = project(L, pose)
    return int(np.sum((np.abs(u) < eps) | (np.abs(u - (L.W - 1)) < eps) |
                      (np.abs(v) < eps) | (np.abs(v - (L.H - 1)) < eps)))


def unpack_h21(H21):
    H21 = np.atleast_2d(H21)
    out = np.zeros((H21.shape[0], 6, 6))
    k = 0
    for a in range(6):
        for b in range(a, 6):
            out[:, a, b] = H21[:, k]
            out[:, b, a] = H21[:, k]
            k += 1
    return out


def rel_frobenius(Hg_a, Hg_b):
    return np.linalg.norm(Hg_a - Hg_b) / max(np.linalg.norm(Hg_b), 1e-300)


def compare_solutions(frame, gpu, orc, tol_m, tol_deg, label=""):
    """Per-hypothesis comparison.  Returns a list of report rows and the
    list of failures (verdict mismatch, or pose error above tolerance for a
    hypothesis converged in both)."""
    gt = frame.gt_pose
    te_g, re_g = S.pose_errors(gpu["poses"], gt)
    te_o, re_o = S.pose_errors(orc["poses"], gt)
    rows, fails = [], []
    for m in range(len(te_g)):
        vg = te_g[m] <= VERDICT_M and re_g[m] <= VERDICT_DEG
        vo = te_o[m] <= VERDICT_M and re_o[m] <= VERDICT_DEG
        dt, dr = S.pose_errors(gpu["poses"][m], orc["poses"][m])
        rows.append((m, vo, vg, float(dt[0]), float(dr[0]), int(orc["status"][m]), int(gpu["status"][m])))
        if vg != vo:
            fails.append((label, m, "verdict", vo, vg, float(dt[0]), float(dr[0])))
        elif vo and (dt[0] > tol_m or dr[0] > tol_deg):
            fails.append((label, m, "pose", float(dt[0]), float(dr[0])))
    return rows, fails


def check_best(frame, gpu, orc, tol_m, tol_deg):
    """The selected hypothesis: same index, or (if two hypotheses reached the
    same minimum) the GPU's pick has the oracle's minimal cost and pose."""
    bg, bo = gpu["best"], orc["best"]
    if bg == bo:
        return True
    if bg < 0 or bo < 0:
        return False
    c = orc["cost"]
    dt, dr = S.pose_errors(orc["poses"][bg], orc["poses"][bo])
    return abs(c[bg] - c[bo]) <= 1e-5 * abs(c[bo]) and dt[0] <= tol_m and dr[0] <= tol_deg
