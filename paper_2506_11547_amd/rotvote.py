"""Thin Python binding of ``librotvote.so`` (argument marshalling only).

PyTorch provides device memory and streams; every step of a solve runs in the
library's HIP kernels.  There is no fallback: if the library is missing or no
GPU is visible, construction raises.

torch is imported before the library is loaded so that the library binds to
the HIP runtime torch already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes as ct
import math
from pathlib import Path

import numpy as np
import torch

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "librotvote.so"
PROBE_PATH = PKG / "librotvote_probe.so"

RV_OK, RV_EINVAL, RV_ENOMEM, RV_EDEVICE, RV_EUNSUPPORTED = 0, -1, -2, -3, -4
RV_EAGAIN, RV_ETIMEDOUT = -5, -6
STATUS_NAMES = {0: "RV_OK", -1: "RV_EINVAL", -2: "RV_ENOMEM", -3: "RV_EDEVICE",
                -4: "RV_EUNSUPPORTED", -5: "RV_EAGAIN", -6: "RV_ETIMEDOUT"}
STRATEGIES = {"auto": 0, "global": 1, "brick": 2, "keys": 3}
STRATEGY_NAMES = {v: k for k, v in STRATEGIES.items()}
FLAG_TIMING = 1
FLAG_BATCH_GRIDS = 2
FLAG_KEEP_HISTOGRAM = 4
MAX_TOPK = 64
NOALLOC_MAX_GRID = 64
NOALLOC_MAX_SAMPLES = 4096
MAX_BATCH_GRID = 64
BATCH_BUCKETS = 4
BATCH_BUCKET_BOUNDS = (512, 2048, 8192)  # n < 512, [512, 2048), [2048, 8192), n >= 8192
MAX_REFINE_ROUNDS = 64
NUM_STAGES = 6
STAGE_NAMES = ("prepare", "vote", "reduce", "topk", "rescore", "mask")

# Names the C header declares; the CPU test suite checks the library exports each.
EXPORTS = ("rot_vote_default_config", "rot_vote_create", "rot_vote_destroy",
           "rot_vote_last_error", "rot_vote_set_stream", "rot_vote_solve", "rot_vote_solve_async",
           "rot_vote_get_histogram", "rot_vote_get_topk", "rot_vote_get_plan",
           "rot_vote_get_timings", "rot_vote_solve_batch", "rot_vote_get_batch_histogram",
           "rot_vote_get_batch_topk", "rot_vote_refine", "rot_vote_solve_multi",
           "rot_vote_get_footprint", "rot_vote_tune", "rot_vote_tune_batch",
           "rot_vote_pairs", "rot_vote_translation", "rot_vote_solve_rigid",
           "rot_vote_server_default_config",
           "rot_vote_server_create",
           "rot_vote_server_destroy", "rot_vote_server_submit", "rot_vote_server_wait",
           "rot_vote_server_stats", "rot_vote_server_last_error", "rot_vote_server_memory",
           "rot_vote_server_pause", "rot_vote_server_request_bytes", "rot_vote_solve_noalloc",
           "rot_vote_solve_batch_async", "rot_vote_set_batch_schedule",
           "rot_vote_get_batch_schedule", "rot_vote_save_tuning", "rot_vote_load_tuning")


class RvConfig(ct.Structure):
    _fields_ = [("device", ct.c_int32), ("stream", ct.c_void_p), ("max_n", ct.c_int64),
                ("max_grid", ct.c_int32), ("samples_per_circle", ct.c_int32),
                ("topk", ct.c_int32), ("vote_strategy", ct.c_int32), ("flags", ct.c_uint32),
                ("max_batch", ct.c_int32), ("batch_brick_edge", ct.c_int32),
                ("reserved", ct.c_int32), ("max_pairs", ct.c_int64)]


class RigidParams(ct.Structure):
    _fields_ = [("mu", ct.c_float), ("eps_rad", ct.c_float), ("grid", ct.c_int32),
                ("refine_rounds", ct.c_int32), ("t_min", ct.c_float), ("t_step", ct.c_float),
                ("t_cells", ct.c_int32), ("t_inlier", ct.c_float)]


class RigidResult(ct.Structure):
    _fields_ = [("q", ct.c_float * 4), ("t", ct.c_float * 3), ("refine_rounds_run", ct.c_int32),
                ("pairs", ct.c_int64), ("rot_inliers", ct.c_int64), ("t_votes", ct.c_int64),
                ("inliers", ct.c_int64)]


class ServerConfig(ct.Structure):
    _fields_ = [("device", ct.c_int32), ("workers", ct.c_int32), ("max_n", ct.c_int64),
                ("max_grid", ct.c_int32), ("topk", ct.c_int32), ("samples_per_circle", ct.c_int32),
                ("max_batch", ct.c_int32), ("batch_max_n", ct.c_int64), ("max_queue", ct.c_int64),
                ("hbm_budget", ct.c_int64), ("reserved", ct.c_int32 * 4)]


REQ_AFTER_STREAM = 1


class Request(ct.Structure):
    _fields_ = [("x", ct.c_void_p), ("y", ct.c_void_p), ("n", ct.c_int64), ("grid", ct.c_int32),
                ("eps_rad", ct.c_float), ("inlier_mask", ct.c_void_p),
                ("refine_rounds", ct.c_int32), ("flags", ct.c_uint32), ("stream", ct.c_void_p)]


class Reply(ct.Structure):
    _fields_ = [("q", ct.c_float * 4), ("inlier_count", ct.c_int64), ("status", ct.c_int32),
                ("batched", ct.c_int32), ("worker", ct.c_int32), ("refine_rounds_run", ct.c_int32),
                ("t_submit", ct.c_double), ("t_start", ct.c_double), ("t_end", ct.c_double),
                ("scratch_bytes", ct.c_int64)]


class RotVoteError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: Path | str = LIB_PATH) -> ct.CDLL:
    """Load (once) and type the C-ABI."""
    global _lib
    if _lib is not None:
        return _lib
    path = Path(path)
    if not path.exists():
        raise ImportError(f"{path.name} is not built; run __graft_entry__.build() first")
    L = ct.CDLL(str(path))
    vp, i32, i64, f32 = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_float
    L.rot_vote_default_config.argtypes = [ct.POINTER(RvConfig)]
    L.rot_vote_default_config.restype = None
    L.rot_vote_create.argtypes = [ct.POINTER(vp), ct.POINTER(RvConfig)]
    L.rot_vote_create.restype = i32
    L.rot_vote_destroy.argtypes = [vp]
    L.rot_vote_destroy.restype = i32
    L.rot_vote_last_error.argtypes = [vp]
    L.rot_vote_last_error.restype = ct.c_char_p
    L.rot_vote_set_stream.argtypes = [vp, vp]
    L.rot_vote_set_stream.restype = i32
    L.rot_vote_solve.argtypes = [vp, vp, vp, i64, i32, f32, ct.POINTER(f32 * 4),
                                 ct.POINTER(i64), vp]
    L.rot_vote_solve.restype = i32
    L.rot_vote_solve_async.argtypes = [vp, vp, vp, i64, i32, f32, vp, vp]
    L.rot_vote_solve_async.restype = i32
    L.rot_vote_solve_noalloc.argtypes = [vp, vp, i64, i32, i32, i32, f32, vp, vp, vp]
    L.rot_vote_solve_noalloc.restype = i32
    L.rot_vote_get_histogram.argtypes = [vp, vp]
    L.rot_vote_get_histogram.restype = i32
    L.rot_vote_get_topk.argtypes = [vp, ct.POINTER(i32), ct.POINTER(i32 * MAX_TOPK),
                                    ct.POINTER(i32 * MAX_TOPK), ct.POINTER(i64 * MAX_TOPK),
                                    ct.POINTER(i32)]
    L.rot_vote_get_topk.restype = i32
    L.rot_vote_get_plan.argtypes = [vp, ct.POINTER(i32), ct.POINTER(i32)]
    L.rot_vote_get_plan.restype = i32
    L.rot_vote_get_timings.argtypes = [vp, ct.POINTER(f32 * NUM_STAGES)]
    L.rot_vote_get_timings.restype = i32
    L.rot_vote_solve_batch.argtypes = [vp, vp, vp, vp, i32, i32, f32, vp, vp, vp]
    L.rot_vote_solve_batch.restype = i32
    L.rot_vote_get_batch_histogram.argtypes = [vp, i32, vp]
    L.rot_vote_get_batch_histogram.restype = i32
    L.rot_vote_get_batch_topk.argtypes = [vp, i32, ct.POINTER(i32), ct.POINTER(i32 * MAX_TOPK),
                                          ct.POINTER(i32 * MAX_TOPK), ct.POINTER(i64 * MAX_TOPK),
                                          ct.POINTER(i32)]
    L.rot_vote_get_batch_topk.restype = i32
    L.rot_vote_refine.argtypes = [vp, vp, vp, i64, f32, i32, ct.POINTER(f32 * 4), ct.POINTER(i64),
                                  vp, ct.POINTER(i32)]
    L.rot_vote_refine.restype = i32
    L.rot_vote_pairs.argtypes = [vp, vp, vp, i64, f32, i64, vp, vp, vp, ct.POINTER(i64)]
    L.rot_vote_pairs.restype = i32
    L.rot_vote_translation.argtypes = [vp, vp, vp, i64, ct.POINTER(f32 * 4), f32, f32, i32, f32,
                                       ct.POINTER(f32 * 3), ct.POINTER(i64), ct.POINTER(i64), vp]
    L.rot_vote_translation.restype = i32
    L.rot_vote_solve_rigid.argtypes = [vp, vp, vp, i64, ct.POINTER(RigidParams),
                                       ct.POINTER(RigidResult), vp]
    L.rot_vote_solve_rigid.restype = i32
    L.rot_vote_solve_multi.argtypes = [vp, vp, vp, i64, i32, f32, i32, f32, i64, ct.POINTER(f32),
                                       ct.POINTER(i64), ct.POINTER(i32), vp]
    L.rot_vote_solve_multi.restype = i32
    L.rot_vote_tune.argtypes = [vp, vp, vp, i64, i32, f32, i32, vp, ct.POINTER(i32),
                                ct.POINTER(f32 * 3)]
    L.rot_vote_tune.restype = i32
    L.rot_vote_tune_batch.argtypes = [vp, vp, vp, ct.POINTER(i64), i32, i32, f32, i32, vp,
                                      ct.POINTER(i32 * BATCH_BUCKETS),
                                      ct.POINTER(f32 * (BATCH_BUCKETS + 1))]
    L.rot_vote_tune_batch.restype = i32
    L.rot_vote_solve_batch_async.argtypes = [vp, vp, vp, i64, vp, i32, i32, f32, vp, vp]
    L.rot_vote_solve_batch_async.restype = i32
    L.rot_vote_set_batch_schedule.argtypes = [vp, i32, ct.POINTER(i32 * BATCH_BUCKETS)]
    L.rot_vote_set_batch_schedule.restype = i32
    L.rot_vote_get_batch_schedule.argtypes = [vp, i32, ct.POINTER(i32 * BATCH_BUCKETS)]
    L.rot_vote_get_batch_schedule.restype = i32
    L.rot_vote_save_tuning.argtypes = [vp, ct.c_char_p]
    L.rot_vote_save_tuning.restype = i32
    L.rot_vote_load_tuning.argtypes = [vp, ct.c_char_p, ct.POINTER(i32)]
    L.rot_vote_load_tuning.restype = i32
    L.rot_vote_get_footprint.argtypes = [vp, ct.POINTER(i64)]
    L.rot_vote_get_footprint.restype = i32
    L.rot_vote_server_default_config.argtypes = [ct.POINTER(ServerConfig)]
    L.rot_vote_server_default_config.restype = None
    L.rot_vote_server_create.argtypes = [ct.POINTER(vp), ct.POINTER(ServerConfig)]
    L.rot_vote_server_create.restype = i32
    L.rot_vote_server_destroy.argtypes = [vp]
    L.rot_vote_server_destroy.restype = i32
    L.rot_vote_server_submit.argtypes = [vp, ct.POINTER(Request), ct.POINTER(ct.c_uint64)]
    L.rot_vote_server_submit.restype = i32
    L.rot_vote_server_wait.argtypes = [vp, ct.c_uint64, i32, ct.POINTER(Reply)]
    L.rot_vote_server_wait.restype = i32
    L.rot_vote_server_stats.argtypes = [vp, ct.POINTER(i32), ct.POINTER(i64), ct.POINTER(i64),
                                        ct.POINTER(i64)]
    L.rot_vote_server_stats.restype = i32
    L.rot_vote_server_memory.argtypes = [vp, ct.POINTER(i64), ct.POINTER(i64), ct.POINTER(i64),
                                         ct.POINTER(i64)]
    L.rot_vote_server_memory.restype = i32
    L.rot_vote_server_pause.argtypes = [vp, i32]
    L.rot_vote_server_pause.restype = i32
    L.rot_vote_server_request_bytes.argtypes = [vp, i64, i32, ct.POINTER(i64)]
    L.rot_vote_server_request_bytes.restype = i32
    L.rot_vote_server_last_error.argtypes = [vp]
    L.rot_vote_server_last_error.restype = ct.c_char_p
    _lib = L
    return L


def _points(x: torch.Tensor, y: torch.Tensor):
    for t, nm in ((x, "x"), (y, "y")):
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda:
            raise ValueError(f"{nm} must be a float32 [3, N] device tensor")
    if x.shape != y.shape:
        raise ValueError("x and y must have the same shape")
    return x.contiguous(), y.contiguous()


def _offsets(offsets) -> np.ndarray:
    """Batch offsets as a contiguous int64 array (no copy when they already are one)."""
    return np.ascontiguousarray(offsets, dtype=np.int64).reshape(-1)


RESULT_BYTES = 32  # sizeof(rv_result): float q[4], int64 count, int32 winner, int32 n_cand


def decode_result(result) -> dict:
    """Reads an rv_result (a uint8 tensor of RESULT_BYTES, device or host).
    Synchronise the stream the solve ran on first: the copy to the host is
    ordered only after torch's current stream."""
    import numpy as np
    b = result.detach().cpu().numpy().astype(np.uint8, copy=False).tobytes()
    if len(b) != RESULT_BYTES:
        raise ValueError(f"an rv_result is {RESULT_BYTES} bytes")
    q = np.frombuffer(b, np.float32, 4, 0)
    count = int(np.frombuffer(b, np.int64, 1, 16)[0])
    winner, n_cand = (int(v) for v in np.frombuffer(b, np.int32, 2, 24))
    return {"q": [float(v) for v in q], "count": count, "winner": winner, "n_cand": n_cand}


def eps_deg_to_rad(eps_deg: float) -> float:
    """Degrees to the float32 radians the C-ABI takes (converted in float64)."""
    return float(ct.c_float(eps_deg * math.pi / 180.0).value)


def solve_noalloc_raw(x_ptr: int, y_ptr: int, n: int, grid: int, eps_rad: float, result_ptr: int,
                      mask_ptr: int, samples_per_circle: int = 0, topk: int = 16,
                      stream: int = 0) -> None:
    """Direct C-ABI call of the handle-free solve that allocates nothing: enqueues
    it on the raw stream and returns; the rv_result at result_ptr is written later."""
    L = load_library()
    st = L.rot_vote_solve_noalloc(ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n, grid,
                                  samples_per_circle, topk, ct.c_float(eps_rad),
                                  ct.c_void_p(stream), ct.c_void_p(result_ptr),
                                  ct.c_void_p(mask_ptr))
    if st != RV_OK:
        raise RotVoteError(st, L.rot_vote_last_error(None).decode())


def solve_noalloc(x: torch.Tensor, y: torch.Tensor, grid: int, eps_deg: float,
                  result: torch.Tensor, mask: torch.Tensor, samples_per_circle: int = 0,
                  topk: int = 16, stream: torch.cuda.Stream | None = None) -> None:
    """The handle-free solve into caller-owned ``result`` (device uint8 of
    RESULT_BYTES) and ``mask`` (device bool [N]) on ``stream`` (default: torch's
    current stream); nothing is allocated, nothing waited for."""
    for t, nm in ((x, "x"), (y, "y")):
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda \
                or not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous float32 [3, N] device tensor")
    if x.shape != y.shape:
        raise ValueError("x and y must have the same shape")
    if result.dtype != torch.uint8 or result.numel() != RESULT_BYTES or not result.is_cuda:
        raise ValueError(f"result must be a device uint8 tensor of {RESULT_BYTES} bytes")
    n = x.shape[1]
    if mask.numel() != n or mask.element_size() != 1 or not mask.is_cuda:
        raise ValueError("mask must be a 1-byte [N] device tensor")
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    solve_noalloc_raw(x.data_ptr(), y.data_ptr(), n, grid, eps_deg_to_rad(eps_deg),
                      result.data_ptr(), mask.data_ptr() if n else 0, samples_per_circle, topk,
                      s.cuda_stream)


class Solver:
    """One library handle: owns the vote grid and scratch for its maxima."""

    def __init__(self, device: int = 0, max_n: int = 1 << 20, max_grid: int = 256,
                 topk: int = 16, samples_per_circle: int = 0, strategy: str = "auto",
                 timing: bool = False, stream: torch.cuda.Stream | None = None,
                 max_batch: int = 0, batch_grids: bool = False, batch_brick_edge: int = 0,
                 max_pairs: int = 0, keep_histogram: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("rotvote needs a HIP GPU; none is visible")
        self._lib = load_library()
        self.device = torch.device("cuda", device)
        cfg = RvConfig()
        self._lib.rot_vote_default_config(ct.byref(cfg))
        cfg.device = device
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg.stream = ct.c_void_p(s.cuda_stream)
        cfg.max_n = max_n
        cfg.max_grid = max_grid
        cfg.samples_per_circle = samples_per_circle
        cfg.topk = topk
        cfg.vote_strategy = STRATEGIES[strategy]
        cfg.flags = ((FLAG_TIMING if timing else 0) | (FLAG_BATCH_GRIDS if batch_grids else 0)
                     | (FLAG_KEEP_HISTOGRAM if keep_histogram else 0))
        cfg.max_batch = max_batch
        cfg.batch_brick_edge = batch_brick_edge
        cfg.max_pairs = max_pairs
        h = ct.c_void_p()
        st = self._lib.rot_vote_create(ct.byref(h), ct.byref(cfg))
        if st != RV_OK:
            raise RotVoteError(st, self._lib.rot_vote_last_error(None).decode())
        self._h = h
        self.topk_k = topk
        self.max_n = max_n
        self.max_grid = max_grid
        self._stream = s
        self._last_grid = None
        self._last_bgrid = None
        self.max_batch = max_batch

    # ---- lifetime
    def close(self):
        if getattr(self, "_h", None):
            self._lib.rot_vote_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int):
        if st != RV_OK:
            raise RotVoteError(st, self._lib.rot_vote_last_error(self._h).decode())

    def set_stream(self, stream: torch.cuda.Stream):
        self._check(self._lib.rot_vote_set_stream(self._h, ct.c_void_p(stream.cuda_stream)))
        self._stream = stream

    # ---- solve
    def solve_raw(self, x_ptr: int, y_ptr: int, n: int, grid: int, eps_rad: float,
                  mask_ptr: int):
        """Direct C-ABI call on raw device addresses; returns (q, count)."""
        q = (ct.c_float * 4)()
        cnt = ct.c_int64()
        self._check(self._lib.rot_vote_solve(self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n,
                                             grid, ct.c_float(eps_rad), ct.byref(q),
                                             ct.byref(cnt), ct.c_void_p(mask_ptr)))
        self._last_grid = grid
        return [q[0], q[1], q[2], q[3]], int(cnt.value)

    def solve(self, x: torch.Tensor, y: torch.Tensor, grid: int, eps_deg: float,
              mask: torch.Tensor | None = None):
        """x, y: float32 [3, N] device tensors (SoA).  Returns (q, count, mask)."""
        for t, nm in ((x, "x"), (y, "y")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda:
                raise ValueError(f"{nm} must be a float32 [3, N] device tensor")
        if x.shape != y.shape:
            raise ValueError("x and y must have the same shape")
        x = x.contiguous()
        y = y.contiguous()
        n = x.shape[1]
        if mask is None:
            mask = torch.empty(n, dtype=torch.bool, device=x.device)
        q, cnt = self.solve_raw(x.data_ptr(), y.data_ptr(), n, grid, eps_deg_to_rad(eps_deg),
                                mask.data_ptr() if n else 0)
        return q, cnt, mask

    def solve_async_raw(self, x_ptr: int, y_ptr: int, n: int, grid: int, eps_rad: float,
                        result_ptr: int, mask_ptr: int):
        """Direct C-ABI call: enqueues the solve on the handle's stream and
        returns at once; the rv_result at result_ptr (device) is written later."""
        self._check(self._lib.rot_vote_solve_async(self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr),
                                                   n, grid, ct.c_float(eps_rad),
                                                   ct.c_void_p(result_ptr), ct.c_void_p(mask_ptr)))
        self._last_grid = grid

    def solve_async(self, x: torch.Tensor, y: torch.Tensor, grid: int, eps_deg: float,
                    result: torch.Tensor | None = None, mask: torch.Tensor | None = None):
        """Enqueues a solve on the handle's stream without waiting.  Returns
        (result, mask): ``result`` is a device uint8 tensor of RESULT_BYTES
        holding an rv_result once the stream has run (``decode_result``)."""
        for t, nm in ((x, "x"), (y, "y")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda:
                raise ValueError(f"{nm} must be a float32 [3, N] device tensor")
            if not t.is_contiguous():
                raise ValueError(f"{nm} must be contiguous (the call does not wait for a copy)")
        if x.shape != y.shape:
            raise ValueError("x and y must have the same shape")
        n = x.shape[1]
        if result is None:
            result = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=x.device)
        if result.dtype != torch.uint8 or result.numel() != RESULT_BYTES or not result.is_cuda:
            raise ValueError(f"result must be a device uint8 tensor of {RESULT_BYTES} bytes")
        if mask is None:
            mask = torch.empty(n, dtype=torch.bool, device=x.device)
        self.solve_async_raw(x.data_ptr(), y.data_ptr(), n, grid, eps_deg_to_rad(eps_deg),
                             result.data_ptr(), mask.data_ptr() if n else 0)
        return result, mask

    def tune(self, x: torch.Tensor, y: torch.Tensor, grid: int, eps_deg: float, reps: int = 3):
        """Measures the vote strategies on this input and fixes the fastest
        for `grid` (AUTO solves).  Returns (strategy name, {name: ms}); -1 ms
        for a strategy the handle cannot run at this grid."""
        x = x.contiguous()
        y = y.contiguous()
        n = x.shape[1]
        scratch = torch.empty(n, dtype=torch.uint8, device=x.device)
        st = ct.c_int32()
        ms = (ct.c_float * 3)()
        self._check(self._lib.rot_vote_tune(self._h, ct.c_void_p(x.data_ptr()),
                                            ct.c_void_p(y.data_ptr()), n, grid,
                                            ct.c_float(eps_deg_to_rad(eps_deg)), reps,
                                            ct.c_void_p(scratch.data_ptr()), ct.byref(st),
                                            ct.byref(ms)))
        return STRATEGY_NAMES[st.value], {"global": ms[0], "brick": ms[1], "keys": ms[2]}

    def solve_multi_raw(self, x_ptr: int, y_ptr: int, n: int, grid: int, eps_rad: float,
                        max_models: int, sep_rad: float, min_inliers: int, labels_ptr: int):
        """Direct C-ABI call; returns (q [M][4], counts [M])."""
        q = (ct.c_float * (4 * max(1, max_models)))()
        cnt = (ct.c_int64 * max(1, max_models))()
        nm = ct.c_int32(-1)
        self._check(self._lib.rot_vote_solve_multi(self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n,
                                                   grid, ct.c_float(eps_rad), max_models,
                                                   ct.c_float(sep_rad), min_inliers, q, cnt,
                                                   ct.byref(nm), ct.c_void_p(labels_ptr)))
        self._last_grid = grid
        m = nm.value
        return [list(q[4 * k:4 * k + 4]) for k in range(m)], [int(c) for c in cnt[:m]]

    def solve_multi(self, x: torch.Tensor, y: torch.Tensor, grid: int, eps_deg: float,
                    max_models: int, sep_deg: float, min_inliers: int,
                    labels: torch.Tensor | None = None):
        """Several rotations from one vote.  Returns (q [M][4], counts [M],
        labels uint8 [N]: 0 unclaimed, m + 1 for model m)."""
        for t, nm in ((x, "x"), (y, "y")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda:
                raise ValueError(f"{nm} must be a float32 [3, N] device tensor")
        if x.shape != y.shape:
            raise ValueError("x and y must have the same shape")
        x = x.contiguous()
        y = y.contiguous()
        n = x.shape[1]
        if labels is None:
            labels = torch.empty(n, dtype=torch.uint8, device=x.device)
        q, cnt = self.solve_multi_raw(x.data_ptr(), y.data_ptr(), n, grid, eps_deg_to_rad(eps_deg),
                                      max_models, math.radians(sep_deg), min_inliers,
                                      labels.data_ptr() if n else 0)
        return q, cnt, labels

    def refine_raw(self, x_ptr: int, y_ptr: int, n: int, eps_rad: float, max_rounds: int,
                   q_in, mask_ptr: int):
        """Direct C-ABI call; the mask at mask_ptr is read and rewritten.
        Returns (q, count, rounds_run)."""
        q = (ct.c_float * 4)(*[float(v) for v in q_in])
        cnt = ct.c_int64()
        rounds = ct.c_int32()
        self._check(self._lib.rot_vote_refine(self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n,
                                              ct.c_float(eps_rad), max_rounds, ct.byref(q),
                                              ct.byref(cnt), ct.c_void_p(mask_ptr),
                                              ct.byref(rounds)))
        return [q[0], q[1], q[2], q[3]], int(cnt.value), int(rounds.value)

    def refine(self, x: torch.Tensor, y: torch.Tensor, q, mask: torch.Tensor, eps_deg: float,
               max_rounds: int = 8):
        """Least-squares refinement (Sec. 4.2) starting from the inlier set
        `mask` (bool/uint8 [N] device tensor, rewritten in place) and the
        rotation q (kept by an ill-posed round).  Returns (q, count, rounds)."""
        for t, nm in ((x, "x"), (y, "y")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda:
                raise ValueError(f"{nm} must be a float32 [3, N] device tensor")
        if x.shape != y.shape or mask.numel() != x.shape[1] or mask.element_size() != 1:
            raise ValueError("x, y must match and mask must be a 1-byte [N] tensor")
        if not mask.is_contiguous():
            raise ValueError("mask must be contiguous (it is rewritten in place)")
        x = x.contiguous()
        y = y.contiguous()
        n = x.shape[1]
        return self.refine_raw(x.data_ptr(), y.data_ptr(), n, eps_deg_to_rad(eps_deg), max_rounds,
                               q, mask.data_ptr() if n else 0)

    # ---- rigid pose (Sec. 4.5)
    def pairs_raw(self, x_ptr: int, y_ptr: int, n: int, mu: float, capacity: int, m_ptr: int,
                  n_ptr: int, idx_ptr: int):
        """Direct C-ABI call; returns (status, P) without raising on RV_ENOMEM."""
        P = ct.c_int64()
        st = self._lib.rot_vote_pairs(self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n,
                                      ct.c_float(mu), capacity, ct.c_void_p(m_ptr),
                                      ct.c_void_p(n_ptr), ct.c_void_p(idx_ptr), ct.byref(P))
        if st not in (RV_OK, RV_ENOMEM):
            self._check(st)
        return st, int(P.value)

    def pairs(self, x: torch.Tensor, y: torch.Tensor, mu: float, capacity: int = 1 << 20):
        """Pairwise differences that pass the length check (Sec. 4.5.1), in
        row order.  Returns (m [3, P], n [3, P], idx int32 [2, P]); the
        buffers are grown to P and the call repeated if P > capacity."""
        x, y = _points(x, y)
        n = x.shape[1]
        while True:
            cap = max(1, int(capacity))
            mo = torch.empty(3 * cap, dtype=torch.float32, device=x.device)
            no = torch.empty(3 * cap, dtype=torch.float32, device=x.device)
            idx = torch.empty(2 * cap, dtype=torch.int32, device=x.device)
            st, P = self.pairs_raw(x.data_ptr(), y.data_ptr(), n, mu, cap, mo.data_ptr(),
                                   no.data_ptr(), idx.data_ptr())
            if st == RV_OK:
                return mo[:3 * P].view(3, P), no[:3 * P].view(3, P), idx[:2 * P].view(2, P)
            capacity = P

    def translation_raw(self, x_ptr: int, y_ptr: int, n: int, q, t_min: float, t_step: float,
                        t_cells: int, t_inlier: float, mask_ptr: int):
        """Direct C-ABI call; returns (t, votes, inliers)."""
        qq = (ct.c_float * 4)(*[float(v) for v in q])
        t = (ct.c_float * 3)()
        votes = ct.c_int64()
        inl = ct.c_int64()
        self._check(self._lib.rot_vote_translation(
            self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n, ct.byref(qq), ct.c_float(t_min),
            ct.c_float(t_step), t_cells, ct.c_float(t_inlier), ct.byref(t), ct.byref(votes),
            ct.byref(inl), ct.c_void_p(mask_ptr)))
        return [t[0], t[1], t[2]], int(votes.value), int(inl.value)

    def translation(self, x: torch.Tensor, y: torch.Tensor, q, t_min: float, t_step: float,
                    t_cells: int, t_inlier: float, mask: torch.Tensor | None = None):
        """Translation vote for a fixed rotation q (Sec. 4.5.2).  Returns
        (t, votes, inliers, mask uint8 [N])."""
        x, y = _points(x, y)
        n = x.shape[1]
        if mask is None:
            mask = torch.empty(n, dtype=torch.uint8, device=x.device)
        t, votes, inl = self.translation_raw(x.data_ptr(), y.data_ptr(), n, q, t_min, t_step,
                                             t_cells, t_inlier, mask.data_ptr() if n else 0)
        return t, votes, inl, mask

    def solve_rigid_raw(self, x_ptr: int, y_ptr: int, n: int, params: RigidParams, mask_ptr: int):
        """Direct C-ABI call; returns the RigidResult."""
        res = RigidResult()
        self._check(self._lib.rot_vote_solve_rigid(self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr),
                                                   n, ct.byref(params), ct.byref(res),
                                                   ct.c_void_p(mask_ptr)))
        return res

    def solve_rigid(self, x: torch.Tensor, y: torch.Tensor, mu: float, grid: int, eps_deg: float,
                    t_min: float, t_step: float, t_cells: int, t_inlier: float,
                    refine_rounds: int = 0, mask: torch.Tensor | None = None):
        """Rigid pose (R, t) from point correspondences (Sec. 4.5).  Returns a
        dict (q, t, pairs, rot_inliers, t_votes, inliers, refine_rounds_run,
        mask uint8 [N])."""
        x, y = _points(x, y)
        n = x.shape[1]
        if mask is None:
            mask = torch.empty(n, dtype=torch.uint8, device=x.device)
        p = RigidParams(mu, eps_deg_to_rad(eps_deg), grid, refine_rounds, t_min, t_step, t_cells,
                        t_inlier)
        r = self.solve_rigid_raw(x.data_ptr(), y.data_ptr(), n, p, mask.data_ptr() if n else 0)
        self._last_grid = grid
        return dict(q=list(r.q), t=list(r.t), pairs=int(r.pairs), rot_inliers=int(r.rot_inliers),
                    t_votes=int(r.t_votes), inliers=int(r.inliers),
                    refine_rounds_run=int(r.refine_rounds_run), mask=mask)

    def tune_batch(self, x: torch.Tensor, y: torch.Tensor, offsets, grid: int, eps_deg: float,
                   reps: int = 2):
        """Chooses the brick edge of each instance-size bucket by measurement on
        this batch and keeps the schedule for `grid`.  Returns (edges per bucket,
        ms: the batch time with 32^3 everywhere, then after trying each bucket at
        16^3, -1 for a bucket without instances)."""
        x = x.contiguous()
        y = y.contiguous()
        B = len(offsets) - 1
        offs = (ct.c_int64 * (B + 1))(*[int(o) for o in offsets])
        scratch = torch.empty(max(1, x.shape[1]), dtype=torch.uint8, device=x.device)
        edges = (ct.c_int32 * BATCH_BUCKETS)()
        ms = (ct.c_float * (BATCH_BUCKETS + 1))()
        self._check(self._lib.rot_vote_tune_batch(self._h, ct.c_void_p(x.data_ptr()),
                                                  ct.c_void_p(y.data_ptr()), offs, B, grid,
                                                  ct.c_float(eps_deg_to_rad(eps_deg)), reps,
                                                  ct.c_void_p(scratch.data_ptr()), ct.byref(edges),
                                                  ct.byref(ms)))
        return list(edges), list(ms)

    def set_batch_schedule(self, grid: int, edges):
        e = (ct.c_int32 * BATCH_BUCKETS)(*[int(v) for v in edges])
        self._check(self._lib.rot_vote_set_batch_schedule(self._h, grid, ct.byref(e)))

    def batch_schedule(self, grid: int) -> list:
        e = (ct.c_int32 * BATCH_BUCKETS)()
        self._check(self._lib.rot_vote_get_batch_schedule(self._h, grid, ct.byref(e)))
        return list(e)

    def save_tuning(self, path):
        self._check(self._lib.rot_vote_save_tuning(self._h, str(path).encode()))

    def load_tuning(self, path) -> int:
        n = ct.c_int32()
        self._check(self._lib.rot_vote_load_tuning(self._h, str(path).encode(), ct.byref(n)))
        return n.value

    def solve_batch_async_raw(self, x_ptr: int, y_ptr: int, n_cols: int, offsets_ptr: int, B: int,
                              grid: int, eps_rad: float, results_ptr: int, mask_ptr: int):
        """Direct C-ABI call: enqueues the device-planned batch on the handle's
        stream and returns; B rv_results are written at results_ptr later."""
        self._check(self._lib.rot_vote_solve_batch_async(
            self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n_cols, ct.c_void_p(offsets_ptr), B,
            grid, ct.c_float(eps_rad), ct.c_void_p(results_ptr), ct.c_void_p(mask_ptr)))
        self._last_bgrid = grid

    def solve_batch_async(self, x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor,
                          grid: int, eps_deg: float, results: torch.Tensor | None = None,
                          mask: torch.Tensor | None = None):
        """Enqueues a batch whose offsets (int64 [B+1]) are a device tensor;
        returns (results uint8 [B, RESULT_BYTES], mask) without waiting."""
        for t, nm in ((x, "x"), (y, "y")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda \
                    or not t.is_contiguous():
                raise ValueError(f"{nm} must be a contiguous float32 [3, N] device tensor")
        if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
            raise ValueError("offsets must be a contiguous int64 device tensor")
        B = offsets.numel() - 1
        if results is None:
            results = torch.empty(max(B, 1), RESULT_BYTES, dtype=torch.uint8, device=x.device)
        if mask is None:
            mask = torch.empty(x.shape[1], dtype=torch.bool, device=x.device)
        self.solve_batch_async_raw(x.data_ptr(), y.data_ptr(), x.shape[1], offsets.data_ptr(), B,
                                   grid, eps_deg_to_rad(eps_deg), results.data_ptr(),
                                   mask.data_ptr() if x.shape[1] else 0)
        return results, mask

    def solve_batch_raw(self, x_ptr: int, y_ptr: int, offsets, grid: int, eps_rad: float,
                        mask_ptr: int):
        """Direct C-ABI call: offsets holds B+1 ints (an int64 array is used
        without a copy).  Returns (q float32 [B, 4], counts int64 [B]) arrays."""
        offs = _offsets(offsets)
        B = offs.shape[0] - 1
        q = np.empty((max(B, 1), 4), np.float32)
        cnt = np.empty(max(B, 1), np.int64)
        self._check(self._lib.rot_vote_solve_batch(self._h, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr),
                                                   ct.c_void_p(offs.ctypes.data), B, grid,
                                                   ct.c_float(eps_rad), ct.c_void_p(q.ctypes.data),
                                                   ct.c_void_p(cnt.ctypes.data),
                                                   ct.c_void_p(mask_ptr)))
        self._last_bgrid = grid
        return q[:B], cnt[:B]

    def solve_batch(self, x: torch.Tensor, y: torch.Tensor, offsets, grid: int, eps_deg: float,
                    mask: torch.Tensor | None = None):
        """Instances are the column ranges [offsets[b], offsets[b+1]) of x, y
        (float32 [3, N] device tensors).  Returns (q float32 [B, 4] and
        counts int64 [B] host arrays, mask)."""
        for t, nm in ((x, "x"), (y, "y")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda:
                raise ValueError(f"{nm} must be a float32 [3, N] device tensor")
        if x.shape != y.shape:
            raise ValueError("x and y must have the same shape")
        offsets = _offsets(offsets)
        if offsets.shape[0] == 0 or offsets[-1] > x.shape[1]:
            raise ValueError("offsets must hold B+1 entries with offsets[B] <= N")
        x = x.contiguous()
        y = y.contiguous()
        n = int(offsets[-1])
        if mask is None:
            mask = torch.empty(x.shape[1], dtype=torch.bool, device=x.device)
        q, cnt = self.solve_batch_raw(x.data_ptr(), y.data_ptr(), offsets, grid,
                                      eps_deg_to_rad(eps_deg), mask.data_ptr() if n else 0)
        return q, cnt, mask

    # ---- test hooks
    def batch_histogram(self, b: int) -> torch.Tensor:
        g = self._last_bgrid
        if g is None:
            raise RuntimeError("no batch yet")
        out = torch.empty(g ** 3, dtype=torch.int32, device=self.device)
        self._check(self._lib.rot_vote_get_batch_histogram(self._h, b, ct.c_void_p(out.data_ptr())))
        return out

    def batch_topk(self, b: int) -> dict:
        nc = ct.c_int32()
        votes = (ct.c_int32 * MAX_TOPK)()
        idx = (ct.c_int32 * MAX_TOPK)()
        inl = (ct.c_int64 * MAX_TOPK)()
        win = ct.c_int32()
        self._check(self._lib.rot_vote_get_batch_topk(self._h, b, ct.byref(nc), ct.byref(votes),
                                                      ct.byref(idx), ct.byref(inl), ct.byref(win)))
        m = nc.value
        return dict(votes=list(votes[:m]), idx=list(idx[:m]), inliers=list(inl[:m]),
                    winner=win.value)

    def histogram(self) -> torch.Tensor:
        """The last solve's vote grid (int32 [G^3], x fastest); the handle must
        have been made with keep_histogram=True (RotVoteError otherwise)."""
        g = self._last_grid
        if g is None:
            raise RuntimeError("no solve yet")
        out = torch.empty(g ** 3, dtype=torch.int32, device=self.device)
        self._check(self._lib.rot_vote_get_histogram(self._h, ct.c_void_p(out.data_ptr())))
        return out

    def topk(self) -> dict:
        nc = ct.c_int32()
        votes = (ct.c_int32 * MAX_TOPK)()
        idx = (ct.c_int32 * MAX_TOPK)()
        inl = (ct.c_int64 * MAX_TOPK)()
        win = ct.c_int32()
        self._check(self._lib.rot_vote_get_topk(self._h, ct.byref(nc), ct.byref(votes),
                                                ct.byref(idx), ct.byref(inl), ct.byref(win)))
        m = nc.value
        return dict(votes=list(votes[:m]), idx=list(idx[:m]), inliers=list(inl[:m]),
                    winner=win.value)

    def plan(self) -> dict:
        J = ct.c_int32()
        s = ct.c_int32()
        self._check(self._lib.rot_vote_get_plan(self._h, ct.byref(J), ct.byref(s)))
        return dict(samples_per_circle=J.value, strategy=STRATEGY_NAMES.get(s.value, s.value))

    def timings(self) -> dict:
        ms = (ct.c_float * NUM_STAGES)()
        self._check(self._lib.rot_vote_get_timings(self._h, ct.byref(ms)))
        return dict(zip(STAGE_NAMES, list(ms)))


class Server:
    """Request server: admission by each request's scratch footprint from one
    device arena (``hbm_budget`` bytes), lanes (a thread, stream and handle
    each) running admitted requests concurrently, batching of small requests.
    Inputs and masks are device tensors the caller keeps alive until the reply
    is collected."""

    def __init__(self, device: int = 0, workers: int = 4, max_n: int = 1 << 20,
                 max_grid: int = 256, topk: int = 16, samples_per_circle: int = 0,
                 max_batch: int = 64, batch_max_n: int = 65536, max_queue: int = 1 << 20,
                 hbm_budget: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("rotvote needs a HIP GPU; none is visible")
        self._lib = load_library()
        torch.cuda.init()
        cfg = ServerConfig()
        self._lib.rot_vote_server_default_config(ct.byref(cfg))
        cfg.device, cfg.workers, cfg.max_n, cfg.max_grid = device, workers, max_n, max_grid
        cfg.topk, cfg.samples_per_circle, cfg.max_batch = topk, samples_per_circle, max_batch
        cfg.batch_max_n, cfg.max_queue, cfg.hbm_budget = batch_max_n, max_queue, hbm_budget
        h = ct.c_void_p()
        st = self._lib.rot_vote_server_create(ct.byref(h), ct.byref(cfg))
        if st != RV_OK:
            raise RotVoteError(st, self._lib.rot_vote_server_last_error(None).decode())
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rot_vote_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit_raw(self, x_ptr: int, y_ptr: int, n: int, grid: int, eps_rad: float, mask_ptr: int,
                   refine_rounds: int = 0, after_stream: int | None = None) -> int:
        """Queues a request on raw device addresses; returns its ticket (raises
        RotVoteError with status RV_EAGAIN when the queue is full).  With
        ``after_stream`` (a raw hipStream_t, 0 for the null stream) the request
        runs after the work already enqueued there."""
        flags = REQ_AFTER_STREAM if after_stream is not None else 0
        r = Request(ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), n, grid, eps_rad, ct.c_void_p(mask_ptr),
                    refine_rounds, flags, ct.c_void_p(after_stream or 0))
        t = ct.c_uint64()
        st = self._lib.rot_vote_server_submit(self._h, ct.byref(r), ct.byref(t))
        if st != RV_OK:
            raise RotVoteError(st, self._lib.rot_vote_server_last_error(self._h).decode())
        return int(t.value)

    def submit(self, x: torch.Tensor, y: torch.Tensor, grid: int, eps_deg: float,
               mask: torch.Tensor, refine_rounds: int = 0,
               stream: torch.cuda.Stream | None = None) -> int:
        """Queues a request; it runs after the work already enqueued on
        ``stream`` (default: torch's current stream), which produced x and y."""
        for t, nm in ((x, "x"), (y, "y")):
            if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda \
                    or not t.is_contiguous():
                raise ValueError(f"{nm} must be a contiguous float32 [3, N] device tensor")
        if x.shape != y.shape or mask.numel() != x.shape[1] or mask.element_size() != 1:
            raise ValueError("x, y must match and mask must be a 1-byte [N] tensor")
        n = x.shape[1]
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        t = self.submit_raw(x.data_ptr(), y.data_ptr(), n, grid, eps_deg_to_rad(eps_deg),
                            mask.data_ptr() if n else 0, refine_rounds, s.cuda_stream)
        self._keep[t] = (x, y, mask)
        return t

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        r = Reply()
        st = self._lib.rot_vote_server_wait(self._h, ticket, timeout_ms, ct.byref(r))
        if st != RV_OK:
            raise RotVoteError(st, self._lib.rot_vote_server_last_error(self._h).decode())
        self._keep.pop(ticket, None)
        return dict(q=list(r.q), count=int(r.inlier_count), status=int(r.status),
                    batched=int(r.batched), worker=int(r.worker),
                    refine_rounds_run=int(r.refine_rounds_run), t_submit=r.t_submit,
                    t_start=r.t_start, t_end=r.t_end, scratch_bytes=int(r.scratch_bytes))

    def stats(self) -> dict:
        w, q, f = ct.c_int32(), ct.c_int64(), ct.c_int64()
        b = ct.c_int64()
        self._lib.rot_vote_server_stats(self._h, ct.byref(w), ct.byref(b), ct.byref(q), ct.byref(f))
        return dict(workers=w.value, device_bytes=b.value, queued=q.value, in_flight=f.value)

    def memory(self) -> dict:
        a, u, p, f = ct.c_int64(), ct.c_int64(), ct.c_int64(), ct.c_int64()
        self._lib.rot_vote_server_memory(self._h, ct.byref(a), ct.byref(u), ct.byref(p),
                                         ct.byref(f))
        return dict(arena_bytes=a.value, in_use=u.value, peak_in_use=p.value,
                    peak_in_flight=f.value)

    def pause(self, paused: bool = True):
        self._lib.rot_vote_server_pause(self._h, int(paused))

    def request_bytes(self, n: int, grid: int) -> int:
        b = ct.c_int64()
        st = self._lib.rot_vote_server_request_bytes(self._h, n, grid, ct.byref(b))
        if st != RV_OK:
            raise RotVoteError(st, self._lib.rot_vote_server_last_error(self._h).decode())
        return b.value


class Probe:
    """Test hooks of ``librotvote_probe.so``: single device steps of the rule."""

    def __init__(self, path: Path | str = PROBE_PATH):
        path = Path(path)
        if not path.exists():
            raise ImportError(f"{path.name} is not built; run __graft_entry__.build() first")
        L = self.lib = ct.CDLL(str(path))
        vp, i64, i32 = ct.c_void_p, ct.c_int64, ct.c_int32
        L.rvp_recip.argtypes = [vp, vp, i64, i32]
        L.rvp_div_sqrt.argtypes = [vp, vp, vp, vp, i64]
        L.rvp_basis.argtypes = [vp, vp, i64, vp, vp, vp]
        L.rvp_cells.argtypes = [vp, i64, i32, vp, i32]
        L.rvp_decode.argtypes = [vp, i64, i32, vp]
        L.rvp_residual.argtypes = [vp, vp, i64, vp, vp]
        L.rvp_table.argtypes = [i32, vp]
        d = ct.POINTER(ct.c_double)
        L.rvp_ceil_valu.argtypes = [i32, i32, d]
        L.rvp_ceil_lds_atomic.argtypes = [i32, i32, i32, d]
        L.rvp_ceil_global_atomic.argtypes = [i64, i32, i32, i32, d]
        L.rvp_ceil_copy.argtypes = [i64, d]
        L.rvp_ceil_read.argtypes = [i64, d]
        for f in (L.rvp_recip, L.rvp_div_sqrt, L.rvp_basis, L.rvp_cells, L.rvp_decode,
                  L.rvp_residual, L.rvp_table, L.rvp_ceil_valu, L.rvp_ceil_lds_atomic,
                  L.rvp_ceil_global_atomic, L.rvp_ceil_copy, L.rvp_ceil_read):
            f.restype = i32

    @staticmethod
    def _p(t: torch.Tensor):
        return ct.c_void_p(t.data_ptr())

    def _run(self, rc: int):
        if rc != 0:
            raise RuntimeError(f"probe kernel failed with HIP error {rc}")

    def recip(self, d: torch.Tensor, fast: bool) -> torch.Tensor:
        torch.cuda.synchronize()
        out = torch.empty_like(d)
        self._run(self.lib.rvp_recip(self._p(d), self._p(out), d.numel(), int(fast)))
        return out

    def div_sqrt(self, a: torch.Tensor, b: torch.Tensor):
        torch.cuda.synchronize()
        q = torch.empty_like(a)
        r = torch.empty_like(a)
        self._run(self.lib.rvp_div_sqrt(self._p(a), self._p(b), self._p(q), self._p(r), a.numel()))
        return q, r

    def basis(self, x: torch.Tensor, y: torch.Tensor):
        torch.cuda.synchronize()
        n = x.shape[1]
        u = torch.empty(n, 4, dtype=torch.float32, device=x.device)
        v = torch.empty_like(u)
        ok = torch.empty(n, dtype=torch.int32, device=x.device)
        self._run(self.lib.rvp_basis(self._p(x), self._p(y), n, self._p(u), self._p(v), self._p(ok)))
        return u, v, ok

    def cells(self, q: torch.Tensor, G: int, fast: bool) -> torch.Tensor:
        torch.cuda.synchronize()
        out = torch.empty(q.shape[0], dtype=torch.int32, device=q.device)
        self._run(self.lib.rvp_cells(self._p(q), q.shape[0], G, self._p(out), int(fast)))
        return out

    def decode(self, idx: torch.Tensor, G: int) -> torch.Tensor:
        torch.cuda.synchronize()
        q = torch.empty(idx.numel(), 4, dtype=torch.float32, device=idx.device)
        self._run(self.lib.rvp_decode(self._p(idx), idx.numel(), G, self._p(q)))
        return q

    def _rate(self, fn, *args) -> float:
        torch.cuda.synchronize()
        r = ct.c_double()
        self._run(fn(*args, ct.byref(r)))
        return r.value

    def ceiling_valu(self, blocks: int = 8192, iters: int = 4096) -> float:
        """32-bit FMA lane-operations per second (independent chains)."""
        return self._rate(self.lib.rvp_ceil_valu, blocks, iters)

    def ceiling_lds_atomic(self, random: bool, blocks: int = 1024, iters: int = 1024) -> float:
        """LDS atomic adds per second (random or bank-distinct cells)."""
        return self._rate(self.lib.rvp_ceil_lds_atomic, blocks, iters, int(random))

    def ceiling_global_atomic(self, cells: int, blocks: int = 4096, iters: int = 256,
                              contiguous: bool = False) -> float:
        """Relaxed device-scope atomic adds per second into an int32 grid of
        ``cells`` entries (a power of two): random cells, or each wave into 64
        consecutive cells."""
        return self._rate(self.lib.rvp_ceil_global_atomic, cells, blocks, iters, int(contiguous))

    def ceiling_copy(self, nbytes: int = 1 << 30) -> float:
        """Bytes read plus written per second by a device copy."""
        return self._rate(self.lib.rvp_ceil_copy, nbytes)

    def ceiling_read(self, nbytes: int = 1 << 30) -> float:
        """Bytes read per second by a streaming read."""
        return self._rate(self.lib.rvp_ceil_read, nbytes)

    def residual(self, x: torch.Tensor, y: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
        torch.cuda.synchronize()
        out = torch.empty(x.shape[1], dtype=torch.float32, device=x.device)
        self._run(self.lib.rvp_residual(self._p(x), self._p(y), x.shape[1], self._p(q),
                                        self._p(out)))
        return out

    def table(self, J: int) -> torch.Tensor:
        """The device-computed sample table of the handle-free solve, float32 [J, 2]."""
        torch.cuda.synchronize()
        out = torch.empty(J, 2, dtype=torch.float32, device="cuda")
        self._run(self.lib.rvp_table(J, self._p(out)))
        return out
