"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU baseline leg
of the benchmark use it; the product path never imports it.

`frame` arguments are duck-typed: anything with the attributes of
`synth.frames.Frame` (levels with H, W, C, feat, K, x, y, z, ref, ref_w,
qconf, iters, loss; poses; dsm.heights/x0/y0/gsd; gravity, range and LM
settings).  Feature values are converted to float64 exactly (bf16 inputs are
passed as their float32 values).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# a test may point the wrapper at a deliberately broken build of oracle.c
_LIB_OVERRIDE = os.environ.get("PILOT_ORACLE_LIB_OVERRIDE")

CONVERGED, MAX_ITERS, STALLED, DEGENERATE, PRUNED = 0, 1, 2, 3, 4

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Level(C.Structure):
    _fields_ = [("H", C.c_int), ("W", C.c_int), ("C", C.c_int),
                ("feat", _dp), ("qconf", _dp),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("N", C.c_int), ("P", _dp), ("ref", _dp), ("ref_w", _dp),
                ("iters", C.c_int), ("loss_kind", C.c_int), ("loss_scale", C.c_double)]


class _Frame(C.Structure):
    _fields_ = [("n_levels", C.c_int), ("lv", _Level * 4),
                ("use_gravity", C.c_int), ("g_imu", C.c_double * 3), ("g_world", C.c_double * 3),
                ("lambda_imu", C.c_double), ("grav_loss_kind", C.c_int), ("grav_loss_scale", C.c_double),
                ("use_range", C.c_int), ("d_range", C.c_double), ("pc", C.c_double * 2),
                ("lambda_range", C.c_double), ("range_loss_kind", C.c_int), ("range_loss_scale", C.c_double),
                ("dsm", _dp), ("Hd", C.c_int), ("Wd", C.c_int),
                ("dsm_x0", C.c_double), ("dsm_y0", C.c_double), ("dsm_gsd", C.c_double),
                ("tau", C.c_double), ("up", C.c_double), ("down", C.c_double),
                ("lam_min_rel", C.c_double), ("lam_max_rel", C.c_double),
                ("tol_t", C.c_double), ("tol_r", C.c_double), ("z_min", C.c_double),
                ("min_valid", C.c_int), ("keep_top", C.c_int), ("prune_level", C.c_int),
                ("adaptive", C.c_int), ("alpha_ratio", C.c_double), ("grav_gate", C.c_double),
                ("range_gate", C.c_double), ("cost_tol", C.c_double)]


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no fast-math; OpenMP over hypotheses)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-fopenmp", "-Wall", "-Wno-unused-function",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB_PATH):
                build()
            L = C.CDLL(_LIB_PATH)
        L.orc_exp.argtypes = [_dp, _dp]
        L.orc_log.argtypes = [_dp, _dp]
        L.orc_compose.argtypes = [_dp, _dp, _dp]
        L.orc_robust.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
        L.orc_bilinear.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_dsm.argtypes = [C.POINTER(_Frame), C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_photo_point.argtypes = [C.POINTER(_Frame), C.c_int, _dp, C.c_int, _dp, _dp, _dp]
        L.orc_photo_point.restype = C.c_int
        L.orc_gravity.argtypes = [C.POINTER(_Frame), _dp, _dp, _dp]
        L.orc_range.argtypes = [C.POINTER(_Frame), _dp, _dp, _dp]
        L.orc_linearize.argtypes = [C.POINTER(_Frame), C.c_int, _dp, _dp, _dp, _dp, _ip]
        L.orc_cholesky_solve6.argtypes = [_dp, _dp, _dp]
        L.orc_cholesky_solve6.restype = C.c_int
        L.orc_linearize_visual.argtypes = [C.POINTER(_Frame), C.c_int, _dp, _dp, _dp, _dp, _ip]
        L.orc_add_priors.argtypes = [C.POINTER(_Frame), _dp, C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_prior_scales.argtypes = [C.POINTER(_Frame), _dp, _dp, _dp]
        L.orc_solve.argtypes = [C.POINTER(_Frame), _dp, C.c_int, C.c_int, _dp, _dp, _ip, _ip, _dp, C.c_int]
        L.orc_solve_alpha.argtypes = [C.POINTER(_Frame), _dp, C.c_int, C.c_int, _dp, _dp, _ip, _ip, _dp, C.c_int,
                                      _dp]
        L.orc_best.argtypes = [_dp, _ip, C.c_int]
        L.orc_best.restype = C.c_int
        L.orc_lift.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp, C.c_int,
                               _dp, C.c_int, C.c_int, C.c_int, C.c_double, _dp, _dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class OracleFrame:
    """Holds float64 copies of a frame's arrays and the C struct that points
    into them (keep this object alive while the struct is used)."""

    def __init__(self, frame):
        self.keep = []
        s = _Frame()
        s.n_levels = len(frame.levels)
        if not 1 <= s.n_levels <= 4:
            raise ValueError("1..4 levels")
        for i, L in enumerate(frame.levels):
            if L.C > 512:
                raise ValueError("oracle supports C <= 512")
            feat = self._k(_f64(L.feat).reshape(-1))
            P = self._k(_f64(np.stack([np.asarray(L.x, np.float64), np.asarray(L.y, np.float64),
                                       np.asarray(L.z, np.float64)], axis=1)).reshape(-1))
            ref = self._k(_f64(L.ref).reshape(-1))
            lv = s.lv[i]
            lv.H, lv.W, lv.C = int(L.H), int(L.W), int(L.C)
            lv.feat = _p(feat)
            lv.qconf = _p(self._k(_f64(L.qconf).reshape(-1))) if getattr(L, "qconf", None) is not None else _dp()
            lv.fx, lv.fy, lv.cx, lv.cy = [float(k) for k in L.K]
            lv.N = int(len(L.x))
            lv.P = _p(P)
            lv.ref = _p(ref)
            lv.ref_w = _p(self._k(_f64(L.ref_w))) if getattr(L, "ref_w", None) is not None else _dp()
            lv.iters = int(L.iters)
            lv.loss_kind, lv.loss_scale = int(L.loss[0]), float(L.loss[1])
        s.use_gravity = int(frame.use_gravity)
        s.g_imu[:] = [float(v) for v in frame.g_imu]
        s.g_world[:] = [float(v) for v in frame.g_world]
        s.lambda_imu = float(frame.lambda_imu)
        s.grav_loss_kind, s.grav_loss_scale = int(frame.gravity_loss[0]), float(frame.gravity_loss[1])
        s.use_range = int(frame.use_range)
        s.d_range = float(frame.d_range)
        s.pc[:] = [float(v) for v in frame.pc]
        s.lambda_range = float(frame.lambda_range)
        s.range_loss_kind, s.range_loss_scale = int(frame.range_loss[0]), float(frame.range_loss[1])
        dsm = self._k(_f64(frame.dsm.heights).reshape(-1))
        s.dsm = _p(dsm)
        s.Hd, s.Wd = frame.dsm.heights.shape
        s.dsm_x0, s.dsm_y0, s.dsm_gsd = float(frame.dsm.x0), float(frame.dsm.y0), float(frame.dsm.gsd)
        lm = frame.lm
        s.tau, s.up, s.down = lm["tau"], lm["up"], lm["down"]
        s.lam_min_rel, s.lam_max_rel = lm["lambda_min_rel"], lm["lambda_max_rel"]
        s.tol_t, s.tol_r, s.z_min = lm["step_tol_t"], lm["step_tol_r"], lm["z_min"]
        s.min_valid = int(lm["min_valid"])
        s.cost_tol = float(lm.get("cost_tol", 0.0))
        s.keep_top = int(getattr(frame, "keep_top", 0))
        s.prune_level = int(getattr(frame, "prune_level", 0))
        s.adaptive = int(getattr(frame, "adaptive_priors", 0))
        s.alpha_ratio = float(getattr(frame, "alpha_ratio", 0.0))
        s.grav_gate = float(getattr(frame, "gravity_gate", 0.0))
        s.range_gate = float(getattr(frame, "range_gate", 0.0))
        self.s = s
        self.ptr = C.pointer(s)

    def _k(self, a):
        self.keep.append(a)
        return a


# ----------------------------------------------------------------------
# thin wrappers
# ----------------------------------------------------------------------
def se3_exp(xi):
    T = np.zeros(12)
    lib().orc_exp(_p(_f64(xi)), _p(T))
    return T


def se3_log(T):
    xi = np.zeros(6)
    lib().orc_log(_p(_f64(T)), _p(xi))
    return xi


def compose(A, B):
    out = np.zeros(12)
    lib().orc_compose(_p(_f64(A)), _p(_f64(B)), _p(out))
    return out


def robust(kind, b, s):
    rho, d = C.c_double(), C.c_double()
    lib().orc_robust(int(kind), float(b), float(s), C.byref(rho), C.byref(d))
    return rho.value, d.value


def bilinear(F, u, v):
    F = _f64(F)
    H, W, Cc = F.shape
    val, du, dv = np.zeros(Cc), np.zeros(Cc), np.zeros(Cc)
    lib().orc_bilinear(_p(F.reshape(-1)), H, W, Cc, float(u), float(v), _p(val), _p(du), _p(dv))
    return val, du, dv


def dsm(of: OracleFrame, x, y):
    h, hx, hy = C.c_double(), C.c_double(), C.c_double()
    lib().orc_dsm(of.ptr, float(x), float(y), C.byref(h), C.byref(hx), C.byref(hy))
    return h.value, hx.value, hy.value


def photo_point(of: OracleFrame, level, T, j):
    Cc = of.s.lv[level].C
    r, J, w = np.zeros(Cc), np.zeros(Cc * 6), C.c_double()
    ok = lib().orc_photo_point(of.ptr, level, _p(_f64(T)), j, _p(r), _p(J), C.byref(w))
    return bool(ok), r, J.reshape(Cc, 6), w.value


def gravity(of: OracleFrame, T):
    r, J = np.zeros(3), np.zeros(18)
    lib().orc_gravity(of.ptr, _p(_f64(T)), _p(r), _p(J))
    return r, J.reshape(3, 6)


def range_term(of: OracleFrame, T):
    r, J = C.c_double(), np.zeros(6)
    lib().orc_range(of.ptr, _p(_f64(T)), C.byref(r), _p(J))
    return r.value, J


def linearize(of: OracleFrame, level, T):
    H, g = np.zeros(36), np.zeros(6)
    c, n = C.c_double(), C.c_int()
    lib().orc_linearize(of.ptr, level, _p(_f64(T)), _p(H), _p(g), C.byref(c), C.byref(n))
    return H.reshape(6, 6), g, c.value, n.value


def linearize_visual(of: OracleFrame, level, T):
    H, g = np.zeros(36), np.zeros(6)
    c, n = C.c_double(), C.c_int()
    lib().orc_linearize_visual(of.ptr, level, _p(_f64(T)), _p(H), _p(g), C.byref(c), C.byref(n))
    return H.reshape(6, 6), g, c.value, n.value


def prior_scales(of: OracleFrame, T, g_vis):
    a = np.zeros(2)
    lib().orc_prior_scales(of.ptr, _p(_f64(T)), _p(_f64(g_vis)), _p(a))
    return a


def cholesky_solve6(A, b):
    x = np.zeros(6)
    rc = lib().orc_cholesky_solve6(_p(_f64(A).reshape(-1)), _p(_f64(b)), _p(x))
    return rc, x


def solve(frame, hyps=None, threads=None, trace=False, of: OracleFrame = None):
    """Run the oracle LM on hypotheses `hyps` (indices, default all; with
    top-K pruning the ranking is among the solved hypotheses).

    Returns dict with poses (k,12), cost (k), iterations (k), status (k),
    alpha (k, 2: gravity and range scales of the last level started),
    best (index into the full hypothesis set among the solved ones, or -1)
    and, with trace=True, trace (k, rows, 4)."""
    of = of or OracleFrame(frame)
    poses = _f64(frame.poses)
    M = poses.shape[0]
    idx = np.arange(M) if hyps is None else np.asarray(hyps, dtype=np.int64)
    sub = np.ascontiguousarray(poses[idx])
    k = len(idx)
    out = np.zeros((k, 12))
    cost = np.zeros(k)
    its = np.zeros(k, dtype=np.int32)
    st = np.zeros(k, dtype=np.int32)
    rows = sum(int(L.iters) for L in frame.levels)
    tr = np.zeros((k, max(rows, 1), 4)) if trace else None
    L = lib()
    L.orc_set_threads(int(threads) if threads else 0)          # 0: all OpenMP threads
    alpha = np.zeros((k, 2))
    L.orc_solve_alpha(of.ptr, _p(sub), 0, k, _p(out), _p(cost), its.ctypes.data_as(_ip),
                      st.ctypes.data_as(_ip), _p(tr) if trace else _dp(), max(rows, 1), _p(alpha))
    b = L.orc_best(_p(cost), st.ctypes.data_as(_ip), k)
    res = dict(poses=out, cost=cost, iterations=its, status=st, alpha=alpha,
               best=int(idx[b]) if b >= 0 else -1, index=idx)
    if trace:
        res["trace"] = tr
    return res


def lift(dsm, x0, y0, gsd, uv, ref_map, scale):
    """Anchors (N, 3) and reference descriptors (N, C) lifted from DSM-crop
    sample coordinates uv (N, 2)."""
    dsm, uv, ref_map = _f64(dsm), _f64(uv), _f64(ref_map)
    Hd, Wd = dsm.shape
    Hr, Wr, Cc = ref_map.shape
    N = uv.shape[0]
    P = np.zeros((N, 3))
    ref = np.zeros((N, Cc))
    lib().orc_lift(_p(dsm.reshape(-1)), Hd, Wd, float(x0), float(y0), float(gsd), _p(uv.reshape(-1)), N,
                   _p(ref_map.reshape(-1)), Hr, Wr, Cc, float(scale), _p(P), _p(ref))
    return P, ref


def threads(n=None):
    """Threads the oracle's solve uses; with n, set them first (0 = all)."""
    if n is not None:
        lib().orc_set_threads(int(n))
    return lib().orc_get_threads()
