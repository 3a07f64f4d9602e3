"""ctypes mirror of include/pilot.h (structs, constants, function table)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PILOT_LIB_OVERRIDE names another build of the same library (the host-sanitized
# copy of build_host_sanitized); by default the in-tree libpilot.so
LIB_PATH = os.environ.get("PILOT_LIB_OVERRIDE") or os.path.join(HERE, "libpilot.so")

MAX_LEVELS = 4
OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
F32, BF16 = 0, 1
LOSS_CAUCHY, LOSS_HUBER, LOSS_L2 = 0, 1, 2
CONVERGED, MAX_ITERS, STALLED, DEGENERATE, PRUNED = 0, 1, 2, 3, 4
FLAG_NO_GRAPH, FLAG_AUTOTUNE, FLAG_PROFILE, FLAG_KEEP_ORDER, FLAG_SORT_ANCHORS = 1, 2, 4, 8, 16

ERROR_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
               EAGAIN: "EAGAIN", EUNSUPPORTED: "EUNSUPPORTED"}

_vp = C.c_void_p
_fp = C.c_void_p
_dp = C.c_void_p


class Config(C.Structure):
    _fields_ = [("device", C.c_int32), ("flags", C.c_int32), ("stream", _vp),
                ("hbm_budget_bytes", C.c_size_t), ("tune_cache", C.c_char_p),
                ("max_slots", C.c_int32), ("reserved", C.c_int32)]


class Level(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("C", C.c_int32), ("dtype", C.c_int32),
                ("feat", _vp), ("qconf", _fp), ("K", C.c_double * 4), ("N", C.c_int32),
                ("x", _fp), ("y", _fp), ("z", _fp), ("ref", _vp), ("ref_w", _fp),
                ("iters", C.c_int32), ("loss_kind", C.c_int32), ("loss_scale", C.c_double)]


class Frame(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("level", Level * MAX_LEVELS), ("M", C.c_int32),
                ("poses_in", _dp),
                ("use_gravity", C.c_int32), ("gravity_loss_kind", C.c_int32),
                ("g_imu", C.c_double * 3), ("g_world", C.c_double * 3),
                ("lambda_imu", C.c_double), ("gravity_loss_scale", C.c_double),
                ("use_range", C.c_int32), ("range_loss_kind", C.c_int32),
                ("d_range", C.c_double), ("pc", C.c_double * 2), ("lambda_range", C.c_double),
                ("range_loss_scale", C.c_double),
                ("dsm", _fp), ("Hd", C.c_int32), ("Wd", C.c_int32),
                ("dsm_x0", C.c_double), ("dsm_y0", C.c_double), ("dsm_gsd", C.c_double),
                ("tau", C.c_double), ("lambda_up", C.c_double), ("lambda_down", C.c_double),
                ("lambda_min_rel", C.c_double), ("lambda_max_rel", C.c_double),
                ("step_tol_t", C.c_double), ("step_tol_r", C.c_double), ("z_min", C.c_double),
                ("min_valid", C.c_int32), ("adaptive_priors", C.c_int32),
                ("prior_poses", _dp), ("prior_best", _vp), ("hyp_offsets", _dp),
                ("keep_top", C.c_int32), ("prune_level", C.c_int32),
                ("alpha_ratio", C.c_double), ("gravity_gate", C.c_double), ("range_gate", C.c_double),
                ("cost_tol", C.c_double)]


class Result(C.Structure):
    _fields_ = [("poses_out", _dp), ("cost", _dp), ("iterations", _vp), ("status", _vp), ("best", _vp),
                ("alpha", _dp)]


class Stats(C.Structure):
    _fields_ = [("pairs", C.c_uint64 * MAX_LEVELS), ("pair_bytes", C.c_uint64 * MAX_LEVELS),
                ("launches", C.c_uint64 * MAX_LEVELS), ("pass_ms", C.c_double * MAX_LEVELS),
                ("timed_launches", C.c_uint64 * MAX_LEVELS),
                ("graph_replays", C.c_uint64), ("graph_captures", C.c_uint64)]


EXPORTS = ["pilot_create", "pilot_destroy", "pilot_last_error", "pilot_solve", "pilot_linearize",
           "pilot_admit_cost", "pilot_admit", "pilot_step", "pilot_poll", "pilot_serving_state",
           "pilot_get_stats", "pilot_autotune", "pilot_tile_choice", "pilot_abi_version", "pilot_sizeof",
           "pilot_sync", "pilot_lift", "pilot_solve_static"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpilot.so (never builds: build first with the package's build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -m paper_2606_31098_amd.build); there is no fallback path")
    L = C.CDLL(path)
    P = C.POINTER
    L.pilot_create.argtypes = [P(_vp), P(Config)]
    L.pilot_destroy.argtypes = [_vp]
    L.pilot_destroy.restype = None
    L.pilot_last_error.argtypes = [_vp]
    L.pilot_last_error.restype = C.c_char_p
    L.pilot_solve.argtypes = [_vp, P(Frame), C.c_int, P(Result)]
    L.pilot_solve_static.argtypes = [_vp, P(Frame), C.c_int, P(Result)]
    L.pilot_linearize.argtypes = [_vp, P(Frame), C.c_int, _vp, _vp, _vp, _vp, _vp]
    L.pilot_admit_cost.argtypes = [_vp, P(Frame), P(C.c_size_t)]
    L.pilot_admit.argtypes = [_vp, P(Frame), P(Result), P(C.c_int)]
    L.pilot_step.argtypes = [_vp]
    L.pilot_poll.argtypes = [_vp, C.c_int]
    L.pilot_serving_state.argtypes = [_vp, P(C.c_int), P(C.c_size_t)]
    L.pilot_sync.argtypes = [_vp]
    L.pilot_lift.argtypes = [_vp, _vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double, _vp, C.c_int32,
                             _vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, _vp, _vp, _vp, _vp]
    L.pilot_get_stats.argtypes = [_vp, P(Stats), C.c_int]
    L.pilot_autotune.argtypes = [_vp, P(Frame)]
    L.pilot_tile_choice.argtypes = [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_char_p, C.c_int]
    L.pilot_abi_version.restype = C.c_int
    L.pilot_sizeof.argtypes = [C.c_char_p]
    L.pilot_sizeof.restype = C.c_size_t
    for name, cls in [("pilot_frame", Frame), ("pilot_level", Level), ("pilot_result", Result),
                      ("pilot_config", Config), ("pilot_stats", Stats)]:
        n = L.pilot_sizeof(name.encode())
        if n != C.sizeof(cls):
            raise RuntimeError(f"ABI mismatch: sizeof({name}) is {n} in the library, {C.sizeof(cls)} here")
    _lib = L
    return L


class PilotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code
