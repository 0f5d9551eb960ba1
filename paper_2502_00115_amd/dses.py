"""Python binding of libdses (the C ABI in include/dses.h).

Argument marshalling only: every step of a registration runs in the HIP
library.  Inputs may be numpy arrays (host memory) or torch CUDA tensors
(device memory, run on the tensor's current stream).  There is no CPU
fallback: without the built library or a gfx950 GPU every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdses.so")

DSES_OK, DSES_E_INVAL, DSES_E_NOCANDIDATE, DSES_E_NOMEM = 0, -1, -2, -3
DSES_E_TIMEOUT, DSES_E_DEVICE, DSES_E_STATE = -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOCANDIDATE", -3: "E_NOMEM", -4: "E_TIMEOUT",
                -5: "E_DEVICE", -6: "E_STATE"}
METRICS = {"trunc_l2": 0, "inliers": 1, "tls": 2, "trunc_l1": 3, "trunc_lp": 4, "votes": 5}
SCORERS = {"auto": 0, "brute": 1, "grid": 2, "df": 3}
DF_LOOKUPS = {"nearest": 0, "trilinear": 1}
DEVICE_PTRS, TIMING, BATCH_TUNE = 0x1, 0x2, 0x4

EXPORTED = [
    "dses_last_error", "dses_init", "dses_version", "dses_kernel_stats", "dses_register",
    "dses_target_create", "dses_target_destroy", "dses_target_field", "dses_rotations_create",
    "dses_rotations_destroy", "dses_register_resident", "dses_register_batch",
    "dses_batch_last_config", "dses_measure_lds_atomics", "dses_rotations_euler",
    "dses_register_exhaustive", "dses_register_noalloc", "dses_noalloc_scratch_bytes",
    "dses_server_create", "dses_server_submit", "dses_server_wait", "dses_server_poll",
    "dses_server_timing", "dses_server_cancel", "dses_server_destroy",
    "dses_debug_fail_allocs",
]


class DsesError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# --------------------------------------------------------------------------
# C structs (mirror include/dses.h)
# --------------------------------------------------------------------------
class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("flags", C.c_uint32), ("delta_t", C.c_float),
                ("tau", C.c_float), ("t_min", C.c_float * 3), ("t_max", C.c_float * 3),
                ("scorer", C.c_int32), ("top_k", C.c_int32), ("stream", C.c_void_p),
                ("records", C.c_void_p), ("topk", C.c_void_p), ("q", C.c_float),
                ("p", C.c_float), ("lane_group", C.c_int32), ("df_lookup", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("rot_index", C.c_int32),
                ("inliers", C.c_int32), ("error", C.c_float), ("votes", C.c_uint32),
                ("n_valid", C.c_int32)]


class KStats(C.Structure):
    _fields_ = [("vote_score_ms", C.c_double), ("score_ms", C.c_double),
                ("select_ms", C.c_double), ("stage_ms", C.c_double),
                ("vote_score_launches", C.c_int64), ("score_launches", C.c_int64),
                ("pairs_voted", C.c_int64), ("pairs_scored", C.c_int64),
                ("candidates", C.c_int64)]


class TargetOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("flags", C.c_uint32), ("df_trunc", C.c_float),
                ("df_res", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("src", C.c_void_p), ("n", C.c_int64), ("tgt", C.c_void_p), ("m", C.c_int64),
                ("rotations", C.c_void_p), ("k", C.c_int64), ("target", C.c_void_p),
                ("rotset", C.c_void_p), ("eps", C.c_float), ("metric", C.c_int32),
                ("delta_t", C.c_float), ("tau", C.c_float), ("t_min", C.c_float * 3),
                ("t_max", C.c_float * 3), ("records", C.c_void_p)]


class BatchOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("flags", C.c_uint32), ("scorer", C.c_int32),
                ("use_graph", C.c_int32), ("tile_rot", C.c_int32), ("vote_parts", C.c_int32),
                ("stream", C.c_void_p), ("df_lookup", C.c_int32)]


class BatchConfig(C.Structure):
    _fields_ = [("items_per_cu", C.c_int32), ("vote_parts", C.c_int32), ("n_items", C.c_int32),
                ("source", C.c_int32), ("candidates", C.c_int32), ("sweep_ms", C.c_float)]


class ServerOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("flags", C.c_uint32),
                ("memory_budget", C.c_int64), ("max_inflight", C.c_int32),
                ("scorer", C.c_int32), ("aging", C.c_float), ("slice_mpairs", C.c_int32)]


RECORD_DTYPE = np.dtype([("bin", "<i4", (3,)), ("votes", "<u4"), ("inliers", "<i4"),
                         ("error", "<f4")])
assert RECORD_DTYPE.itemsize == 24
CANDIDATE_DTYPE = np.dtype([("rot_index", "<i4"), ("inliers", "<i4"), ("error", "<f4"),
                            ("votes", "<u4"), ("t", "<f4", (3,))])
assert CANDIDATE_DTYPE.itemsize == 28
TOPK_MAX = 64

_lib = None


def lib():
    """Load libdses.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DsesError(DSES_E_DEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, f, u32 = C.c_void_p, C.c_int64, C.c_int32, C.c_float, C.c_uint32
        L.dses_last_error.restype = C.c_char_p
        L.dses_version.restype = C.c_char_p
        L.dses_init.argtypes = [i32]
        L.dses_kernel_stats.argtypes = [C.POINTER(KStats), i32]
        L.dses_register.argtypes = [vp, i64, vp, i64, vp, i64, f, i32, C.POINTER(Options),
                                    C.POINTER(Result)]
        L.dses_target_create.argtypes = [vp, i64, C.POINTER(TargetOpts), C.POINTER(vp)]
        L.dses_target_destroy.argtypes = [vp]
        L.dses_target_field.argtypes = [vp, vp, vp, vp]
        L.dses_rotations_create.argtypes = [vp, i64, u32, C.POINTER(vp)]
        L.dses_rotations_destroy.argtypes = [vp]
        L.dses_register_resident.argtypes = [vp, vp, vp, i64, f, i32, C.POINTER(Options),
                                             C.POINTER(Result)]
        L.dses_batch_last_config.argtypes = [C.POINTER(BatchConfig)]
        L.dses_rotations_euler.argtypes = [vp, i32, f, vp]
        L.dses_register_exhaustive.argtypes = [vp, i64, vp, i64, vp, i64, f, i32,
                                               C.POINTER(Options), C.POINTER(Result)]
        L.dses_register_noalloc.argtypes = [vp, i64, vp, i64, vp, i64, f, i32,
                                            C.POINTER(Options), C.POINTER(Result)]
        L.dses_measure_lds_atomics.argtypes = [i32, C.POINTER(C.c_double),
                                               C.POINTER(C.c_double)]
        L.dses_register_batch.argtypes = [C.POINTER(Problem), i32, C.POINTER(BatchOpts),
                                          C.POINTER(Result), C.POINTER(i32)]
        L.dses_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(vp)]
        L.dses_server_submit.argtypes = [vp, vp, vp, vp, i64, f, i32, C.POINTER(Options),
                                         C.POINTER(C.c_uint64)]
        L.dses_server_wait.argtypes = [vp, C.c_uint64, i32, C.POINTER(Result), C.POINTER(i32),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.dses_server_cancel.argtypes = [vp, C.c_uint64]
        L.dses_server_poll.argtypes = [vp, C.c_uint64]
        L.dses_server_poll.restype = i32
        L.dses_server_timing.argtypes = [vp, C.c_uint64, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]
        L.dses_server_destroy.argtypes = [vp]
        L.dses_debug_fail_allocs.argtypes = [i32, i32]
        for name in EXPORTED:
            if name not in ("dses_last_error", "dses_version", "dses_noalloc_scratch_bytes"):
                getattr(L, name).restype = i32
        L.dses_noalloc_scratch_bytes.restype = C.c_size_t
        _lib = L
    return _lib


def _check(status):
    if status != DSES_OK:
        raise DsesError(status, lib().dses_last_error().decode())


def last_error() -> str:
    return lib().dses_last_error().decode()


def init(device: int = 0):
    _check(lib().dses_init(device))


def version() -> str:
    return lib().dses_version().decode()


@dataclass
class Registration:
    R: np.ndarray
    t: np.ndarray
    rot_index: int
    inliers: int
    error: float
    votes: int
    n_valid: int
    records: np.ndarray | None = None
    top: np.ndarray | None = None          # CANDIDATE_DTYPE, best first (top_k > 0)
    queue_s: float | None = None           # served requests: submission -> admission
    total_s: float | None = None           # served requests: submission -> completion


def _result(r: Result, records=None, top=None) -> Registration:
    return Registration(np.array(r.R, np.float32).reshape(3, 3), np.array(r.t, np.float32),
                        int(r.rot_index), int(r.inliers), float(r.error), int(r.votes),
                        int(r.n_valid), records, top)


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Args:
    """Turns numpy arrays or torch tensors into pointers; keeps them alive."""

    def __init__(self):
        self.keep = []
        self.device = None

    def ptr(self, x, cols):
        if x is None:
            return None, 0
        if _is_torch(x):
            import torch
            if not x.is_cuda:
                x = x.detach().to(torch.float32).contiguous().numpy()
            else:
                if x.dtype != torch.float32 or not x.is_contiguous():
                    raise ValueError("device tensors must be contiguous float32")
                if x.numel() % cols:
                    raise ValueError(f"expected rows of {cols} floats")
                if self.device is False:
                    raise ValueError("mix of host arrays and device tensors")
                self.device = True
                self.keep.append(x)
                return C.c_void_p(x.data_ptr()), x.numel() // cols
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        if a.size % cols:
            raise ValueError(f"expected rows of {cols} floats")
        if self.device is True:
            raise ValueError("mix of host arrays and device tensors")
        self.device = False
        self.keep.append(a)
        return C.c_void_p(a.ctypes.data), a.size // cols


def _stream_of(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _options(args: _Args, delta_t, tau, t_min, t_max, scorer, timing, stream, records_ptr,
             q=0.0, lp=0.0, lane_group=0, df_lookup="nearest"):
    o = Options()
    o.q = float(q)
    o.p = float(lp)
    o.lane_group = int(lane_group)
    o.df_lookup = DF_LOOKUPS[df_lookup]
    o.struct_size = C.sizeof(Options)
    o.flags = (DEVICE_PTRS if args.device else 0) | (TIMING if timing else 0)
    o.delta_t = 0.0 if delta_t is None else float(delta_t)
    o.tau = 0.0 if tau is None else float(tau)
    if t_min is not None or t_max is not None:
        lo = np.broadcast_to(np.asarray(-1.0 if t_min is None else t_min, np.float32), 3)
        hi = np.broadcast_to(np.asarray(1.0 if t_max is None else t_max, np.float32), 3)
        o.t_min[:] = [float(v) for v in lo]
        o.t_max[:] = [float(v) for v in hi]
    o.scorer = SCORERS[scorer]
    o.stream = _stream_of(stream) if args.device else None
    o.records = records_ptr
    return o


def _records_buffer(args: _Args, k: int):
    if args.device:
        import torch
        buf = torch.empty(k * RECORD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        args.keep.append(buf)
        return buf, C.c_void_p(buf.data_ptr())
    buf = np.zeros(k, RECORD_DTYPE)
    args.keep.append(buf)
    return buf, C.c_void_p(buf.ctypes.data)


def _records_out(buf, dtype=RECORD_DTYPE):
    if isinstance(buf, np.ndarray):
        return buf
    return np.frombuffer(buf.cpu().numpy().tobytes(), dtype)


def _topk_buffer(args: _Args, k: int, o: Options):
    """Caller-owned top-k array for k candidates (device memory for device inputs)."""
    if not 0 <= k <= TOPK_MAX:
        raise ValueError(f"top_k must be in 0..{TOPK_MAX}")
    if k == 0:
        return None
    if args.device:
        import torch
        buf = torch.empty(k * CANDIDATE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        ptr = buf.data_ptr()
    else:
        buf = np.zeros(k, CANDIDATE_DTYPE)
        ptr = buf.ctypes.data
    args.keep.append(buf)
    o.top_k = k
    o.topk = C.c_void_p(ptr)
    return buf


def register(src, tgt, rotations, eps, metric="trunc_l2", *, delta_t=None, tau=None,
             t_min=None, t_max=None, scorer="auto", records=False, top_k=0, q=0.0,
             lp=0.0, timing=False, stream=None, lane_group=0,
             df_lookup="nearest") -> Registration:
    """dses_register: the full sweep over the rotation list (top_k > 0: also the best
    top_k candidates in selection order, Registration.top; q > 0: score only the
    rotations with M_k >= q M*; lp: exponent of metric "trunc_lp"; lane_group: vote
    layout, 16, 32 or 64 reference points per lane group, 0 automatic)."""
    args = _Args()
    ps, n = args.ptr(src, 3)
    pt, m = args.ptr(tgt, 3)
    pr, k = args.ptr(rotations, 9)
    rbuf, rptr = _records_buffer(args, k) if records else (None, None)
    o = _options(args, delta_t, tau, t_min, t_max, scorer, timing, stream, rptr, q, lp,
                 lane_group, df_lookup)
    tbuf = _topk_buffer(args, int(top_k), o)
    res = Result()
    _check(lib().dses_register(ps, n, pt, m, pr, k, C.c_float(eps), METRICS[metric],
                               C.byref(o), C.byref(res)))
    return _result(res, _records_out(rbuf) if records else None,
                   _records_out(tbuf, CANDIDATE_DTYPE) if tbuf is not None else None)


def register_noalloc(src, tgt, rotations, eps, metric="trunc_l2", *, delta_t=None, tau=None,
                     t_min=None, t_max=None, scorer="auto", records=False, lp=0.0,
                     stream=None, lane_group=0) -> Registration:
    """dses_register_noalloc: dses_register on device tensors with every device buffer
    taken from the library's static scratch array (no allocation in the call; the
    records buffer, when asked for, is allocated here by torch, outside the call)."""
    args = _Args()
    ps, n = args.ptr(src, 3)
    pt, m = args.ptr(tgt, 3)
    pr, k = args.ptr(rotations, 9)
    if not args.device:
        raise ValueError("register_noalloc takes device tensors")
    rbuf, rptr = _records_buffer(args, k) if records else (None, None)
    o = _options(args, delta_t, tau, t_min, t_max, scorer, False, stream, rptr, 0.0, lp,
                 lane_group, "nearest")
    res = Result()
    _check(lib().dses_register_noalloc(ps, n, pt, m, pr, k, C.c_float(eps), METRICS[metric],
                                       C.byref(o), C.byref(res)))
    return _result(res, _records_out(rbuf) if records else None)


def noalloc_scratch_bytes() -> int:
    return int(lib().dses_noalloc_scratch_bytes())


def debug_fail_allocs(skip: int, count: int) -> None:
    """dses_debug_fail_allocs: of the library's next allocations the first `skip`
    succeed and the `count` after them fail; (0, 0) turns the injection off."""
    _check(lib().dses_debug_fail_allocs(int(skip), int(count)))


def register_exhaustive(src, tgt, rotations, eps, metric="trunc_l2", *, delta_t=None, tau=None,
                        t_min=None, t_max=None, scorer="auto", records=False, lp=0.0,
                        timing=False, stream=None) -> Registration:
    """dses_register_exhaustive: Alg. 1 over the rotation list and the box lattice."""
    args = _Args()
    ps, n = args.ptr(src, 3)
    pt, m = args.ptr(tgt, 3)
    pr, k = args.ptr(rotations, 9)
    rbuf, rptr = _records_buffer(args, k) if records else (None, None)
    o = _options(args, delta_t, tau, t_min, t_max, scorer, timing, stream, rptr, 0.0, lp)
    res = Result()
    _check(lib().dses_register_exhaustive(ps, n, pt, m, pr, k, C.c_float(eps), METRICS[metric],
                                          C.byref(o), C.byref(res)))
    return _result(res, _records_out(rbuf) if records else None)


def kernel_stats(reset=False) -> dict:
    s = KStats()
    _check(lib().dses_kernel_stats(C.byref(s), int(bool(reset))))
    return {name: getattr(s, name) for name, _ in KStats._fields_}


class Target:
    """A reference cloud resident in device memory (optionally with a distance field)."""

    def __init__(self, tgt, df_trunc: float = 0.0, df_res: int = 0):
        args = _Args()
        p, m = args.ptr(tgt, 3)
        o = TargetOpts(C.sizeof(TargetOpts), DEVICE_PTRS if args.device else 0,
                       float(df_trunc), int(df_res))
        h = C.c_void_p()
        _check(lib().dses_target_create(p, m, C.byref(o), C.byref(h)))
        self.handle, self.m, self.df_res = h, m, (df_res or 128) if df_trunc > 0 else 0

    def field(self):
        n = self.df_res
        fld = np.zeros((n, n, n), np.float32)
        lo = np.zeros(3, np.float32)
        h = np.zeros(3, np.float32)
        _check(lib().dses_target_field(self.handle, fld.ctypes.data, lo.ctypes.data,
                                       h.ctypes.data))
        return fld, lo, h

    def close(self):
        if self.handle:
            lib().dses_target_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RotationSet:
    """A rotation list resident in device memory."""

    def __init__(self, rotations):
        args = _Args()
        p, k = args.ptr(rotations, 9)
        h = C.c_void_p()
        _check(lib().dses_rotations_create(p, k, DEVICE_PTRS if args.device else 0, C.byref(h)))
        self.handle, self.k = h, k

    def close(self):
        if self.handle:
            lib().dses_rotations_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def register_resident(target: Target, rotset: RotationSet, src, eps, metric="trunc_l2", *,
                      delta_t=None, tau=None, t_min=None, t_max=None, scorer="auto",
                      records=False, top_k=0, q=0.0, lp=0.0, timing=False,
                      stream=None, df_lookup="nearest") -> Registration:
    args = _Args()
    ps, n = args.ptr(src, 3)
    rbuf, rptr = _records_buffer(args, rotset.k) if records else (None, None)
    o = _options(args, delta_t, tau, t_min, t_max, scorer, timing, stream, rptr, q, lp,
                 df_lookup=df_lookup)
    tbuf = _topk_buffer(args, int(top_k), o)
    res = Result()
    _check(lib().dses_register_resident(target.handle, rotset.handle, ps, n, C.c_float(eps),
                                        METRICS[metric], C.byref(o), C.byref(res)))
    return _result(res, _records_out(rbuf) if records else None,
                   _records_out(tbuf, CANDIDATE_DTYPE) if tbuf is not None else None)


def register_batch(problems, *, scorer="auto", use_graph=True, tile_rot=0, vote_parts=0,
                   autotune=False, records=False, timing=False, stream=None,
                   df_lookup="nearest"):
    """dses_register_batch over dicts with keys src, tgt/target, rotations/rotset, eps,
    and optionally metric, delta_t, tau, t_min, t_max.  Returns (results, statuses).
    autotune=True sets DSES_BATCH_TUNE (time candidate launch layouts on this batch and
    keep the fastest for its class); batch_last_config() reports the layout used."""
    args = _Args()
    arr = (Problem * len(problems))()
    bufs = []
    for i, pb in enumerate(problems):
        P = arr[i]
        P.src, P.n = args.ptr(pb["src"], 3)
        if pb.get("target") is not None:
            P.target, P.m = pb["target"].handle, pb["target"].m
        else:
            P.tgt, P.m = args.ptr(pb["tgt"], 3)
        if pb.get("rotset") is not None:
            P.rotset, P.k = pb["rotset"].handle, pb["rotset"].k
        else:
            P.rotations, P.k = args.ptr(pb["rotations"], 9)
        P.eps = float(pb["eps"])
        P.metric = METRICS[pb.get("metric", "trunc_l2")]
        P.delta_t = float(pb.get("delta_t") or 0.0)
        P.tau = float(pb.get("tau") or 0.0)
        if pb.get("t_min") is not None:
            P.t_min[:] = [float(v) for v in np.broadcast_to(pb["t_min"], 3)]
            P.t_max[:] = [float(v) for v in np.broadcast_to(pb["t_max"], 3)]
        if records:
            b, ptr = _records_buffer(args, int(P.k))
            bufs.append(b)
            P.records = ptr
        else:
            bufs.append(None)
    o = BatchOpts(C.sizeof(BatchOpts), (DEVICE_PTRS if args.device else 0) |
                  (TIMING if timing else 0) | (BATCH_TUNE if autotune else 0), SCORERS[scorer],
                  int(bool(use_graph)), int(tile_rot), int(vote_parts),
                  _stream_of(stream) if args.device else None, DF_LOOKUPS[df_lookup])
    res = (Result * len(problems))()
    st = (C.c_int32 * len(problems))()
    _check(lib().dses_register_batch(arr, len(problems), C.byref(o), res, st))
    out = [_result(res[i], _records_out(bufs[i]) if records else None)
           if st[i] == DSES_OK else None for i in range(len(problems))]
    return out, [int(v) for v in st]


def measure_lds_atomics(pattern: str = "random") -> dict:
    """LDS atomic throughput of the device (dses_measure_lds_atomics)."""
    a, b = C.c_double(), C.c_double()
    _check(lib().dses_measure_lds_atomics({"conflict_free": 0, "random": 1}[pattern],
                                          C.byref(a), C.byref(b)))
    return {"adds_per_s": a.value, "per_cu_per_cycle": b.value}


def euler_grid(K: int, step: float, center=None) -> np.ndarray:
    """Alg. 2's Euler rotation grid ((2K+1)^3 x 9 float32, dses_rotations_euler)."""
    side = 2 * int(K) + 1
    out = np.zeros((side ** 3, 9), np.float32)
    c = None if center is None else np.ascontiguousarray(np.asarray(center, np.float32).reshape(9))
    _check(lib().dses_rotations_euler(None if c is None else c.ctypes.data, int(K),
                                      C.c_float(step), out.ctypes.data))
    return out


def batch_last_config() -> dict:
    """Launch layout of this thread's last dses_register_batch (dses_batch_last_config)."""
    cfg = BatchConfig()
    _check(lib().dses_batch_last_config(C.byref(cfg)))
    source = {0: "default", 1: "tuned", 2: "tuned-cache", 3: "caller"}[cfg.source]
    return {"items_per_cu": cfg.items_per_cu, "vote_parts": cfg.vote_parts,
            "n_items": cfg.n_items, "source": source, "candidates": cfg.candidates,
            "sweep_ms": cfg.sweep_ms}


class Server:
    """Continuous-batching registration server (dses_server_*)."""

    def __init__(self, memory_budget=0, max_inflight=0, scorer="auto", aging=0.0,
                 slice_mpairs=0):
        o = ServerOpts(C.sizeof(ServerOpts), 0, int(memory_budget), int(max_inflight),
                       SCORERS[scorer], float(aging), int(slice_mpairs))
        h = C.c_void_p()
        _check(lib().dses_server_create(C.byref(o), C.byref(h)))
        self.handle = h
        self._pending = {}

    def submit(self, target: Target, rotset: RotationSet, src, eps, metric="trunc_l2", *,
               delta_t=None, tau=None, t_min=None, t_max=None, scorer=None,
               df_lookup="nearest", records=False, top_k=0) -> int:
        """Queue a request (host source); per-request options as dses_server_submit
        describes.  records / top_k buffers are kept here until wait() returns them."""
        a = np.ascontiguousarray(np.asarray(src, np.float32).reshape(-1, 3))
        args = _Args()
        args.device = False
        rbuf, rptr = _records_buffer(args, rotset.k) if records else (None, None)
        o = _options(args, delta_t, tau, t_min, t_max, scorer or "auto", False, None, rptr,
                     df_lookup=df_lookup)
        if scorer is None:
            o.scorer = 0
        tbuf = _topk_buffer(args, int(top_k), o)
        rid = C.c_uint64()
        _check(lib().dses_server_submit(self.handle, target.handle, rotset.handle,
                                        a.ctypes.data, len(a), C.c_float(eps), METRICS[metric],
                                        C.byref(o), C.byref(rid)))
        self._pending[int(rid.value)] = (args, rbuf, tbuf)
        return int(rid.value)

    def wait(self, req_id: int, timeout_ms: int = -1) -> Registration:
        """Result of a request (consumes it); .queue_s / .total_s are its latencies."""
        res = Result()
        st = C.c_int32()
        q, t = C.c_double(), C.c_double()
        _check(lib().dses_server_wait(self.handle, req_id, timeout_ms, C.byref(res),
                                      C.byref(st), C.byref(q), C.byref(t)))
        _, rbuf, tbuf = self._pending.pop(req_id, (None, None, None))
        _check(st.value)
        out = _result(res, rbuf, tbuf)
        out.queue_s, out.total_s = q.value, t.value
        return out

    def poll(self, req_id: int) -> int:
        return int(lib().dses_server_poll(self.handle, req_id))

    def timing(self, req_id: int):
        """(queue_s, total_s) of a finished request not yet consumed by wait()."""
        q, t = C.c_double(), C.c_double()
        _check(lib().dses_server_timing(self.handle, req_id, C.byref(q), C.byref(t)))
        return q.value, t.value

    def cancel(self, req_id: int):
        """Withdraw a request still in the queue (raises E_STATE once it is admitted)."""
        _check(lib().dses_server_cancel(self.handle, req_id))
        self._pending.pop(req_id, None)

    def close(self):
        if self.handle:
            lib().dses_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
