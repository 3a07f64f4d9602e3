"""Python binding of libpilot: argument marshalling only.

PyTorch provides device memory and the stream; every step of the solve runs
in the library's HIP kernels.  There is no CPU path: without the built
library (or without a GPU) these calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi as A
from ._abi import PilotError

__all__ = ["Context", "DeviceFrame", "DeviceResult", "PilotError"]


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class DeviceFrame:
    """Device copies of one frame's inputs and the pilot_frame pointing at them.

    `frame` is duck-typed like synth.frames.Frame (levels with H, W, C, feat,
    K, x, y, z, ref, ref_w, qconf, iters, loss; poses; dsm; priors; lm).
    dtype 'bf16' rounds feat and ref to bfloat16 (round-to-nearest-even) on
    the device, once.
    """

    def __init__(self, frame, device: str = "cuda", dtype: str = "f32", share_points: bool = True,
                 poses: Optional[np.ndarray] = None, prior: Optional["torch.Tensor"] = None,
                 prior_best: Optional["torch.Tensor"] = None, hyp_offsets: Optional[np.ndarray] = None):
        self.frame = frame
        self.keep: List[torch.Tensor] = []
        s = A.Frame()
        s.n_levels = len(frame.levels)
        prev_xyz = None
        for i, L in enumerate(frame.levels):
            lv = s.level[i]
            lv.H, lv.W, lv.C = int(L.H), int(L.W), int(L.C)
            tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
            lv.dtype = A.BF16 if dtype == "bf16" else A.F32
            feat = self._k(torch.as_tensor(np.ascontiguousarray(L.feat), dtype=torch.float32).to(device).to(tdt).contiguous())
            ref = self._k(torch.as_tensor(np.ascontiguousarray(L.ref), dtype=torch.float32).to(device).to(tdt).contiguous())
            lv.feat = feat.data_ptr()
            lv.ref = ref.data_ptr()
            lv.qconf = _ptr(self._k(torch.as_tensor(L.qconf, dtype=torch.float32).to(device).contiguous())) \
                if getattr(L, "qconf", None) is not None else None
            lv.K[:] = [float(k) for k in L.K]
            lv.N = int(len(L.x))
            xyz = (np.asarray(L.x), np.asarray(L.y), np.asarray(L.z))
            if share_points and prev_xyz is not None and all(np.array_equal(a, b[0]) for a, b in zip(xyz, prev_xyz)):
                tx, ty, tz = [t for _, t in prev_xyz]
            else:
                tx, ty, tz = [self._k(torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).to(device)) for a in xyz]
            prev_xyz = list(zip(xyz, (tx, ty, tz)))
            lv.x, lv.y, lv.z = tx.data_ptr(), ty.data_ptr(), tz.data_ptr()
            lv.ref_w = _ptr(self._k(torch.as_tensor(L.ref_w, dtype=torch.float32).to(device))) \
                if getattr(L, "ref_w", None) is not None else None
            lv.iters = int(L.iters)
            lv.loss_kind, lv.loss_scale = int(L.loss[0]), float(L.loss[1])
        if hyp_offsets is not None:
            # hypotheses generated on the device around `prior` (row prior_best)
            off = self._k(torch.as_tensor(np.ascontiguousarray(hyp_offsets, dtype=np.float64)).to(device))
            s.M = int(off.shape[0])
            s.hyp_offsets = off.data_ptr()
            s.prior_poses = self._k(prior.to(device=device, dtype=torch.float64).contiguous()).data_ptr()
            s.prior_best = _ptr(self._k(prior_best)) if prior_best is not None else None
            s.poses_in = None
            self.poses = None
        else:
            P = np.ascontiguousarray(frame.poses if poses is None else poses, dtype=np.float64)
            self.poses = self._k(torch.as_tensor(P).to(device))
            s.M = int(P.shape[0])
            s.poses_in = self.poses.data_ptr()
        s.use_gravity = int(frame.use_gravity)
        s.gravity_loss_kind = int(frame.gravity_loss[0])
        s.gravity_loss_scale = float(frame.gravity_loss[1])
        s.g_imu[:] = [float(v) for v in frame.g_imu]
        s.g_world[:] = [float(v) for v in frame.g_world]
        s.lambda_imu = float(frame.lambda_imu)
        s.use_range = int(frame.use_range)
        s.range_loss_kind = int(frame.range_loss[0])
        s.range_loss_scale = float(frame.range_loss[1])
        s.d_range = float(frame.d_range)
        s.pc[:] = [float(v) for v in frame.pc]
        s.lambda_range = float(frame.lambda_range)
        dsm = self._k(torch.as_tensor(np.ascontiguousarray(frame.dsm.heights), dtype=torch.float32).to(device))
        s.dsm = dsm.data_ptr()
        s.Hd, s.Wd = frame.dsm.heights.shape
        s.dsm_x0, s.dsm_y0, s.dsm_gsd = float(frame.dsm.x0), float(frame.dsm.y0), float(frame.dsm.gsd)
        lm = frame.lm
        s.tau, s.lambda_up, s.lambda_down = lm["tau"], lm["up"], lm["down"]
        s.lambda_min_rel, s.lambda_max_rel = lm["lambda_min_rel"], lm["lambda_max_rel"]
        s.step_tol_t, s.step_tol_r, s.z_min = lm["step_tol_t"], lm["step_tol_r"], lm["z_min"]
        s.min_valid = int(lm["min_valid"])
        s.cost_tol = float(lm.get("cost_tol", 0.0))
        s.keep_top = int(getattr(frame, "keep_top", 0))
        s.prune_level = int(getattr(frame, "prune_level", 0))
        s.adaptive_priors = int(getattr(frame, "adaptive_priors", 0))
        s.alpha_ratio = float(getattr(frame, "alpha_ratio", 0.0))
        s.gravity_gate = float(getattr(frame, "gravity_gate", 0.0))
        s.range_gate = float(getattr(frame, "range_gate", 0.0))
        self.s = s

    def _k(self, t: torch.Tensor) -> torch.Tensor:
        self.keep.append(t)
        return t

    @property
    def M(self) -> int:
        return int(self.s.M)

    def input_bytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in self.keep)


class DeviceResult:
    def __init__(self, M: int, device: str = "cuda"):
        self.poses = torch.empty((M, 12), dtype=torch.float64, device=device)
        self.cost = torch.empty(M, dtype=torch.float64, device=device)
        self.iterations = torch.empty(M, dtype=torch.int32, device=device)
        self.status = torch.empty(M, dtype=torch.int32, device=device)
        self.best = torch.empty(1, dtype=torch.int32, device=device)
        self.alpha = torch.empty((M, 2), dtype=torch.float64, device=device)
        self.s = A.Result(self.poses.data_ptr(), self.cost.data_ptr(), self.iterations.data_ptr(),
                          self.status.data_ptr(), self.best.data_ptr(), self.alpha.data_ptr())

    def numpy(self) -> dict:
        return dict(poses=self.poses.cpu().numpy(), cost=self.cost.cpu().numpy(),
                    iterations=self.iterations.cpu().numpy(), status=self.status.cpu().numpy(),
                    alpha=self.alpha.cpu().numpy(), best=int(self.best.cpu().item()))


@dataclass
class Stats:
    pairs: list
    pair_bytes: list
    launches: list
    pass_ms: list
    timed_launches: list
    graph_replays: int
    graph_captures: int


class Context:
    """A pilot_ctx bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None, flags: int = 0,
                 hbm_budget_bytes: int = 0, tune_cache: Optional[str] = None, max_slots: int = 0):
        self.lib = A.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libpilot needs a GPU: torch.cuda.is_available() is False")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        cfg = A.Config(device, flags, C.c_void_p(self.stream.cuda_stream), hbm_budget_bytes,
                       tune_cache.encode() if tune_cache else None, max_slots, 0)
        h = C.c_void_p()
        rc = self.lib.pilot_create(C.byref(h), C.byref(cfg))
        if rc != A.OK:
            raise PilotError(rc, self.lib.pilot_last_error(None).decode())
        self.h = h

    def _check(self, rc: int):
        if rc != A.OK and rc < 0:
            raise PilotError(rc, self.lib.pilot_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.pilot_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.lib.pilot_last_error(self.h).decode()

    # ------------------------------------------------------------------ solve
    def solve(self, frames: Sequence[DeviceFrame], results: Optional[Sequence[DeviceResult]] = None):
        n = len(frames)
        if results is None:
            results = [DeviceResult(f.M, f"cuda:{self.device}") for f in frames]
        fa = (A.Frame * n)(*[f.s for f in frames])
        ra = (A.Result * n)(*[r.s for r in results])
        self._check(self.lib.pilot_solve(self.h, fa, n, ra))
        return results

    def solve_static(self, frames: Sequence[DeviceFrame], results: Optional[Sequence[DeviceResult]] = None):
        """pilot_solve_static: the solve on the library's fixed device scratch
        (no device allocation; tiles from the tile database or heuristic)."""
        n = len(frames)
        if results is None:
            results = [DeviceResult(f.M, f"cuda:{self.device}") for f in frames]
        fa = (A.Frame * n)(*[f.s for f in frames])
        ra = (A.Result * n)(*[r.s for r in results])
        self._check(self.lib.pilot_solve_static(self.h, fa, n, ra))
        return results

    def solve_raw(self, frame_array, n, result_array):
        """Solve from prebuilt ctypes arrays (used by timing loops)."""
        return self._check(self.lib.pilot_solve(self.h, frame_array, n, result_array))

    def linearize(self, frame: DeviceFrame, level: int, poses: torch.Tensor):
        M = frame.M
        dev = poses.device
        poses = poses.to(torch.float64).contiguous()
        H = torch.empty((M, 21), dtype=torch.float64, device=dev)
        g = torch.empty((M, 6), dtype=torch.float64, device=dev)
        cost = torch.empty(M, dtype=torch.float64, device=dev)
        n = torch.empty(M, dtype=torch.int32, device=dev)
        self._check(self.lib.pilot_linearize(self.h, C.byref(frame.s), level, poses.data_ptr(), H.data_ptr(),
                                             g.data_ptr(), cost.data_ptr(), n.data_ptr()))
        return H, g, cost, n

    def lift(self, dsm: torch.Tensor, x0: float, y0: float, gsd: float, uv: torch.Tensor, ref_map: torch.Tensor,
             scale: float, points: bool = True):
        """Lift anchors at DSM-crop coordinates uv (N, 2) and sample their
        reference descriptors from ref_map (Hr, Wr, C; f32 or bf16).
        Returns (x, y, z, ref) device tensors (x, y, z None if points=False)."""
        dsm = dsm.to(torch.float32).contiguous()
        uv = uv.to(torch.float32).contiguous()
        ref_map = ref_map.contiguous()
        N = int(uv.shape[0])
        Hr, Wr, Cc = ref_map.shape
        dt = A.BF16 if ref_map.dtype == torch.bfloat16 else A.F32
        dev = uv.device
        x = y = z = None
        if points:
            x, y, z = [torch.empty(N, dtype=torch.float32, device=dev) for _ in range(3)]
        ref = torch.empty((N, Cc), dtype=ref_map.dtype, device=dev)
        self._check(self.lib.pilot_lift(self.h, dsm.data_ptr(), dsm.shape[0], dsm.shape[1], float(x0), float(y0),
                                        float(gsd), uv.data_ptr(), N, ref_map.data_ptr(), Hr, Wr, Cc, dt,
                                        float(scale), _ptr(x), _ptr(y), _ptr(z), ref.data_ptr()))
        return x, y, z, ref

    def autotune(self, frame: DeviceFrame):
        self._check(self.lib.pilot_autotune(self.h, C.byref(frame.s)))

    def tile_choice(self, C_: int, dtype: int, N: int, M: int, HW: int) -> str:
        buf = C.create_string_buffer(128)
        self._check(self.lib.pilot_tile_choice(self.h, C_, dtype, N, M, HW, buf, 128))
        return buf.value.decode()

    def stats(self, reset: bool = False) -> Stats:
        st = A.Stats()
        self._check(self.lib.pilot_get_stats(self.h, C.byref(st), 1 if reset else 0))
        return Stats(list(st.pairs), list(st.pair_bytes), list(st.launches), list(st.pass_ms),
                     list(st.timed_launches), st.graph_replays, st.graph_captures)

    # ---------------------------------------------------------------- serving
    def admit_cost(self, frame: DeviceFrame) -> int:
        n = C.c_size_t()
        self._check(self.lib.pilot_admit_cost(self.h, C.byref(frame.s), C.byref(n)))
        return n.value

    def admit(self, frame: DeviceFrame, result: DeviceResult) -> Optional[int]:
        """Slot index, or None when no slot/budget is free (EAGAIN)."""
        slot = C.c_int(-1)
        rc = self.lib.pilot_admit(self.h, C.byref(frame.s), C.byref(result.s), C.byref(slot))
        if rc == A.EAGAIN:
            return None
        self._check(rc)
        return slot.value

    def step(self):
        self._check(self.lib.pilot_step(self.h))

    def poll(self, slot: int) -> bool:
        return self._check(self.lib.pilot_poll(self.h, slot)) == 1

    def sync(self):
        self._check(self.lib.pilot_sync(self.h))

    def serving_state(self):
        a, b = C.c_int(), C.c_size_t()
        self._check(self.lib.pilot_serving_state(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value


def unpack_h21(H21: np.ndarray) -> np.ndarray:
    """(M, 21) upper-triangle rows -> (M, 6, 6) symmetric."""
    H21 = np.atleast_2d(H21)
    out = np.zeros((H21.shape[0], 6, 6))
    k = 0
    for a in range(6):
        for b in range(a, 6):
            out[:, a, b] = H21[:, k]
            out[:, b, a] = H21[:, k]
            k += 1
    return out
