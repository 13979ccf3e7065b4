"""ctypes binding of the C ABI in include/tina_pfb.h.

Argument marshalling only: every step of the filter bank runs in the HIP
library.  torch supplies device memory (tensor data pointers) and streams.
If libtina_pfb.so is missing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtina_pfb.so")

SAMPLE = {"r32": 0, "c64": 1}
WINDOW = {"rect": 0, "hann": 1, "hamming": 2, "blackman": 3, "custom": 4}
PRECISION = {"fp32": 0, "bf16": 1, "bf16x3": 2, "fp16": 3, "fp16x3": 4, "fp8": 5, "mxfp8": 6}
OUTPUT = {"pfb": 0, "fir": 1, "inverse": 2}
DFT = {"dense": 0, "factored": 1, "fused": 2, "compensated": 3, "table": 4}

STATUS = {0: "OK", 1: "INVALID_ARGUMENT", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY", 4: "DEVICE",
          5: "BUSY", 6: "NOT_READY", 7: "TOO_LARGE", 8: "TIMEOUT", 9: "CANCELLED"}

# Every symbol include/tina_pfb.h (and the other public headers) declare.
EXPORTS = [
    "tina_last_error", "tina_version",
    "tina_pfb_plan", "tina_pfb_plan_destroy", "tina_pfb_channels_out", "tina_pfb_plan_taps",
    "tina_pfb_output_frames", "tina_pfb_execute", "tina_pfb_execute_noalloc", "tina_pfb_synthesize",
    "tina_pfb_state_create", "tina_pfb_state_destroy", "tina_pfb_state_reset", "tina_pfb_state_size",
    "tina_pfb_state_export", "tina_pfb_state_import",
    "tina_pfb_profile_enable", "tina_pfb_profile_read",
    "tina_pfb_batch_create", "tina_pfb_batch_destroy", "tina_pfb_batch_execute", "tina_pfb_batch_tune",
    "tina_pfb_batch_split_units",
    "tina_server_create", "tina_server_destroy", "tina_server_stream_create", "tina_pfb_submit", "tina_pfb_poll",
    "tina_pfb_wait", "tina_pfb_cancel", "tina_server_get_stats", "tina_server_arena_simulate",
    "tina_server_schedule_simulate",
    "tina_unfold", "tina_fir_create", "tina_fir_destroy", "tina_fir_execute",
]


class TinaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Work(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("state", ctypes.c_void_p), ("d_in", ctypes.c_void_p),
                ("n_samples", ctypes.c_int64), ("d_out", ctypes.c_void_p),
                ("out_capacity_frames", ctypes.c_int64), ("frames_written", ctypes.c_int64)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("device", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_streams", ctypes.c_int32), ("max_active", ctypes.c_int32), ("max_queued", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("frames_per_step", ctypes.c_int64),
                ("use_graph", ctypes.c_int32), ("max_channels", ctypes.c_int32),
                ("dft_algorithm", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("stream_id", ctypes.c_int32), ("flags", ctypes.c_int32), ("host_in", ctypes.c_void_p),
                ("n_samples", ctypes.c_int64), ("host_out", ctypes.c_void_p),
                ("out_capacity_frames", ctypes.c_int64), ("ready_stream", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pad_", ctypes.c_int32), ("frames", ctypes.c_int64),
                ("t_submit_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_first_step_us", ctypes.c_double), ("t_done_us", ctypes.c_double),
                ("steps", ctypes.c_int32), ("pad2_", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("samples", ctypes.c_int64), ("frames", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("admitted", ctypes.c_int64), ("admission_waits", ctypes.c_int64),
                ("device_busy_ms", ctypes.c_double), ("now_us", ctypes.c_double),
                ("arena_in_use", ctypes.c_int64), ("arena_high_water", ctypes.c_int64)]


class _SchedOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("arg", ctypes.c_int32), ("value", ctypes.c_int64)]


class _SchedEvent(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("status", ctypes.c_int32), ("id", ctypes.c_uint64),
                ("a", ctypes.c_int64), ("b", ctypes.c_int64)]


SCHED = {"add_stream": 1, "submit": 2, "admit": 3, "ready": 4, "step": 5, "complete": 6, "cancel": 7}
SCHED_NAME = {v: k for k, v in SCHED.items()}


class _Desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("channels", ctypes.c_int32), ("taps", ctypes.c_int32),
                ("sample_type", ctypes.c_int32), ("window", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("output", ctypes.c_int32), ("device", ctypes.c_int32),
                ("custom_taps", ctypes.POINTER(ctypes.c_double)), ("workspace_bytes", ctypes.c_int64),
                ("dft_algorithm", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "tina_last_error": ([], ctypes.c_char_p),
        "tina_version": ([], ctypes.c_char_p),
        "tina_pfb_plan": ([ctypes.POINTER(_Desc), ctypes.POINTER(vp)], i32),
        "tina_pfb_plan_destroy": ([vp], i32),
        "tina_pfb_channels_out": ([vp, P64], i32),
        "tina_pfb_plan_taps": ([vp, vp], i32),
        "tina_pfb_output_frames": ([vp, vp, i64, P64], i32),
        "tina_pfb_execute": ([vp, vp, i64, vp, i64, vp, P64, vp], i32),
        "tina_pfb_execute_noalloc": ([vp, vp, i64, vp, i64, vp, P64, vp], i32),
        "tina_pfb_synthesize": ([vp, vp, i64, vp, i64, vp, P64, vp], i32),
        "tina_pfb_state_create": ([vp, ctypes.POINTER(vp)], i32),
        "tina_pfb_state_destroy": ([vp], i32),
        "tina_pfb_state_reset": ([vp], i32),
        "tina_pfb_state_size": ([vp, P64, P64], i32),
        "tina_pfb_state_export": ([vp, vp, i64, P64], i32),
        "tina_pfb_state_import": ([vp, vp, i64], i32),
        "tina_pfb_profile_enable": ([vp, i32], i32),
        "tina_pfb_profile_read": ([vp, ctypes.POINTER(ctypes.c_double), P64, ctypes.POINTER(ctypes.c_double), P64], i32),
        "tina_pfb_batch_create": ([i32, i32, i32, i64, ctypes.POINTER(vp)], i32),
        "tina_pfb_batch_destroy": ([vp], i32),
        "tina_pfb_batch_split_units": ([vp, vp, i32, vp], i32),
        "tina_server_create": ([ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)], i32),
        "tina_server_destroy": ([vp], i32),
        "tina_server_stream_create": ([vp, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_int32)], i32),
        "tina_pfb_submit": ([vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)], i32),
        "tina_pfb_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(_Result)], i32),
        "tina_pfb_wait": ([vp, ctypes.c_uint64, i64, ctypes.POINTER(_Result)], i32),
        "tina_pfb_cancel": ([vp, ctypes.c_uint64], i32),
        "tina_server_get_stats": ([vp, ctypes.POINTER(_ServerStats)], i32),
        "tina_server_arena_simulate": ([i64, vp, i32, vp, P64], i32),
        "tina_server_schedule_simulate": ([i32, i32, i64, i64, ctypes.POINTER(_SchedOp), i32,
                                           ctypes.POINTER(_SchedEvent), i32, ctypes.POINTER(ctypes.c_int32)], i32),
        "tina_unfold": ([vp, i64, i64, i64, vp, i64, P64, vp], i32),
        "tina_fir_create": ([i32, vp, i32, i32, ctypes.POINTER(vp)], i32),
        "tina_fir_destroy": ([vp], i32),
        "tina_fir_execute": ([vp, vp, i64, vp, vp], i32),
        "tina_pfb_batch_execute": ([vp, ctypes.POINTER(_Work), i32, vp], i32),
        "tina_pfb_batch_tune": ([vp, ctypes.POINTER(_Work), i32, vp, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes, fn.restype = args, res
    _lib = lib
    return lib


def check(status: int):
    if status != 0:
        raise TinaError(status, load().tina_last_error().decode())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def check_device_tensor(t, what: str, dtype, ndim: int, device: int, cols=None):
    """Raise ValueError unless t is a contiguous torch tensor of `dtype` with
    `ndim` dimensions (and `cols` columns) on cuda:`device`: the C ABI takes
    raw pointers, so a wrong type or layout would be read or written out of
    bounds."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if t.dim() != ndim:
        raise ValueError(f"{what} must have {ndim} dimension(s), got shape {tuple(t.shape)}")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{what} must have {cols} columns, got shape {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{what} must be on cuda:{device}, got {t.device}")


def check_host_array(a, what: str, dtype, ndim: int, cols=None):
    """Raise ValueError unless a is a C-contiguous numpy array of `dtype` with
    `ndim` dimensions (and `cols` columns)."""
    if not isinstance(a, np.ndarray):
        raise ValueError(f"{what} must be a numpy array or a CUDA tensor, got {type(a).__name__}")
    if a.dtype != np.dtype(dtype):
        raise ValueError(f"{what} must be {np.dtype(dtype)}, got {a.dtype}")
    if a.ndim != ndim:
        raise ValueError(f"{what} must have {ndim} dimension(s), got shape {a.shape}")
    if cols is not None and a.shape[1] != cols:
        raise ValueError(f"{what} must have {cols} columns, got shape {a.shape}")
    if not a.flags.c_contiguous:
        raise ValueError(f"{what} must be C-contiguous")


class Plan:
    """A filter-bank plan: P channels, M taps per branch, a prototype window,
    the sample type, the DFT precision form and the output kind."""

    def __init__(self, channels: int, taps: int, sample_type: str = "r32", window: str = "hann",
                 precision: str = "fp32", output: str = "pfb", device: int = 0, custom_taps=None,
                 workspace_bytes: int = 0, dft: str = "dense"):
        lib = load()
        self.P, self.M = int(channels), int(taps)
        self.sample_type, self.precision, self.output = sample_type, precision, output
        self.complex_input = sample_type == "c64"
        d = _Desc()
        d.struct_size = ctypes.sizeof(_Desc)
        d.channels, d.taps = self.P, self.M
        d.sample_type, d.window = SAMPLE[sample_type], WINDOW[window]
        d.precision, d.output, d.device = PRECISION[precision], OUTPUT[output], int(device)
        d.workspace_bytes = int(workspace_bytes)
        d.dft_algorithm = DFT[dft]
        self._custom = None
        if custom_taps is not None:
            self._custom = np.ascontiguousarray(custom_taps, dtype=np.float64)
            d.custom_taps = self._custom.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        check(lib.tina_pfb_plan(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        check(lib.tina_pfb_channels_out(self.handle, ctypes.byref(n)))
        self.channels_out = n.value
        self.device = int(device)

    def close(self):
        if getattr(self, "handle", None):
            load().tina_pfb_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Enable (and clear) or disable per-stage HIP-event timing."""
        check(load().tina_pfb_profile_enable(self.handle, int(bool(enable))))

    def profile_read(self):
        """(fir_ms_total, fir_launches, dft_ms_total, dft_launches) since enable."""
        a, b = ctypes.c_double(), ctypes.c_double()
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        check(load().tina_pfb_profile_read(self.handle, ctypes.byref(a), ctypes.byref(na), ctypes.byref(b),
                                           ctypes.byref(nb)))
        return a.value, na.value, b.value, nb.value

    def taps(self) -> np.ndarray:
        h = np.empty(self.P * self.M, dtype=np.float64)
        check(load().tina_pfb_plan_taps(self.handle, h.ctypes.data_as(ctypes.c_void_p)))
        return h

    def output_frames(self, n_samples: int, state: "State | None" = None) -> int:
        f = ctypes.c_int64()
        check(load().tina_pfb_output_frames(self.handle, state.handle if state else None, int(n_samples),
                                            ctypes.byref(f)))
        return f.value

    def out_shape(self, frames: int):
        return (frames, self.channels_out)

    def alloc_out(self, frames: int):
        import torch
        if self.output == "fir":
            dt = torch.complex64 if self.complex_input else torch.float32
        else:
            dt = torch.complex64
        return torch.empty((frames, self.channels_out), dtype=dt, device=f"cuda:{self.device}")

    def execute(self, x, out=None, state: "State | None" = None, stream=None, noalloc: bool = False):
        """Run on a 1-D device tensor x (float32 or complex64); returns the
        output tensor (frames x channels_out).  noalloc=True calls
        tina_pfb_execute_noalloc (the library's static scratch instead of the
        plan's workspace; pass `out` too so nothing is allocated here)."""
        import torch
        want = torch.complex64 if self.complex_input else torch.float32
        check_device_tensor(x, "input", want, 1, self.device)
        n = x.numel()
        frames = self.output_frames(n, state)
        if out is None:
            out = self.alloc_out(frames)
        out_dt = want if self.output == "fir" else torch.complex64
        check_device_tensor(out, "out", out_dt, 2, self.device, cols=self.channels_out)
        cap = out.shape[0]
        fw = ctypes.c_int64()
        fn = load().tina_pfb_execute_noalloc if noalloc else load().tina_pfb_execute
        check(fn(self.handle, ctypes.c_void_p(x.data_ptr() if n else 0), n,
                                      ctypes.c_void_p(out.data_ptr() if out.numel() else 0), cap,
                                      state.handle if state else None, ctypes.byref(fw), _stream_handle(stream)))
        return out[: fw.value]

    __call__ = execute

    def synthesize(self, X, out=None, state: "State | None" = None, stream=None):
        """Synthesis bank of an output="inverse" plan: X (frames x P complex64
        device tensor) -> frames * P complex64 samples."""
        import torch
        check_device_tensor(X, "X", torch.complex64, 2, self.device, cols=self.P)
        F = X.shape[0]
        if out is None:
            out = torch.empty(F * self.P, dtype=torch.complex64, device=X.device)
        check_device_tensor(out, "out", torch.complex64, 1, self.device)
        n = ctypes.c_int64()
        check(load().tina_pfb_synthesize(self.handle, ctypes.c_void_p(X.data_ptr() if F else 0), F,
                                         ctypes.c_void_p(out.data_ptr() if out.numel() else 0), out.numel(),
                                         state.handle if state else None, ctypes.byref(n), _stream_handle(stream)))
        return out[: n.value]


class State:
    """Per-stream filter state (history and residue) on the device."""

    def __init__(self, plan: Plan):
        self.plan = plan
        h = ctypes.c_void_p()
        check(load().tina_pfb_state_create(plan.handle, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().tina_pfb_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        check(load().tina_pfb_state_reset(self.handle))

    def size(self):
        n, r = ctypes.c_int64(), ctypes.c_int64()
        check(load().tina_pfb_state_size(self.handle, ctypes.byref(n), ctypes.byref(r)))
        return n.value, r.value

    def export(self) -> np.ndarray:
        n, _ = self.size()
        dt = np.complex64 if self.plan.complex_input else np.float32
        buf = np.empty(n, dtype=dt)
        got = ctypes.c_int64()
        check(load().tina_pfb_state_export(self.handle, buf.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(got)))
        return buf[: got.value]

    def load_from(self, buf: np.ndarray):
        dt = np.complex64 if self.plan.complex_input else np.float32
        b = np.ascontiguousarray(buf, dtype=dt)
        check(load().tina_pfb_state_import(self.handle, b.ctypes.data_as(ctypes.c_void_p), b.size))


class Batch:
    """Batched execution: many (plan, input, output, state) chunks per call,
    one persistent launch per stage."""

    def __init__(self, precision: str = "fp32", max_items: int = 256, workspace_bytes: int = 1 << 30,
                 device: int = 0):
        h = ctypes.c_void_p()
        check(load().tina_pfb_batch_create(int(device), PRECISION[precision], int(max_items), int(workspace_bytes),
                                           ctypes.byref(h)))
        self.handle = h
        self.precision = precision

    def close(self):
        if getattr(self, "handle", None):
            load().tina_pfb_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _works(items):
        import torch
        arr = (_Work * max(1, len(items)))()
        for i, it in enumerate(items):
            plan, x, out = it[0], it[1], it[2]
            state = it[3] if len(it) > 3 else None
            want = torch.complex64 if plan.complex_input else torch.float32
            check_device_tensor(x, f"item {i} input", want, 1, plan.device)
            check_device_tensor(out, f"item {i} out", torch.complex64, 2, plan.device, cols=plan.channels_out)
            w = arr[i]
            w.plan = plan.handle.value
            w.state = state.handle.value if state is not None else None
            w.d_in = x.data_ptr() if x.numel() else None
            w.n_samples = x.numel()
            w.d_out = out.data_ptr() if out.numel() else None
            w.out_capacity_frames = out.shape[0]
        return arr

    def execute(self, items, stream=None):
        """items: list of (plan, x, out[, state]); returns frames written per item."""
        arr = self._works(items)
        check(load().tina_pfb_batch_execute(self.handle, arr, len(items), _stream_handle(stream)))
        return [arr[i].frames_written for i in range(len(items))]

    def tune(self, items, stream=None):
        """Autotune launch shapes on this batch shape; returns (fir_tf_mult, gemm_tile_n)."""
        arr = self._works(items)
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(load().tina_pfb_batch_tune(self.handle, arr, len(items), _stream_handle(stream), ctypes.byref(a),
                                         ctypes.byref(b)))
        return a.value, b.value


def split_units(units, cost):
    """Cost-balanced split of a stage's units into 8 contiguous XCD ranges
    (host-only helper of the batched launch); returns 9 bounds."""
    u = np.ascontiguousarray(units, dtype=np.int64)
    c = np.ascontiguousarray(cost, dtype=np.float64)
    b = np.zeros(9, dtype=np.int64)
    check(load().tina_pfb_batch_split_units(u.ctypes.data_as(ctypes.c_void_p), c.ctypes.data_as(ctypes.c_void_p),
                                            len(u), b.ctypes.data_as(ctypes.c_void_p)))
    return b


def arena_simulate(capacity: int, ops):
    """Run the server's arena allocator on the host (no device): see
    tina_server_arena_simulate.  Returns (per-op results, bytes in use)."""
    o = np.ascontiguousarray(ops, dtype=np.int64)
    out = np.zeros(len(o), dtype=np.int64)
    used = ctypes.c_int64()
    check(load().tina_server_arena_simulate(int(capacity), o.ctypes.data_as(ctypes.c_void_p), len(o),
                                            out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(used)))
    return out, used.value


class Server:
    """Continuous-batching channelizer server (one thread, one device)."""

    def __init__(self, precision: str = "fp32", max_streams: int = 64, max_active: int = 32, max_queued: int = 4096,
                 hbm_budget_bytes: int = 8 << 30, frames_per_step: int = 256, use_graph: bool = False,
                 max_channels: int = 4096, device: int = 0, dft: str = "dense"):
        c = _ServerConfig()
        c.struct_size = ctypes.sizeof(_ServerConfig)
        c.device, c.precision = int(device), PRECISION[precision]
        c.max_streams, c.max_active, c.max_queued = int(max_streams), int(max_active), int(max_queued)
        c.hbm_budget_bytes, c.frames_per_step = int(hbm_budget_bytes), int(frames_per_step)
        c.use_graph, c.max_channels = int(bool(use_graph)), int(max_channels)
        c.dft_algorithm = DFT[dft]
        h = ctypes.c_void_p()
        check(load().tina_server_create(ctypes.byref(c), ctypes.byref(h)))
        self.handle = h
        self.device = int(device)
        self._streams = {}
        self._lent = {}   # request id -> (input, output) kept alive until done

    def close(self):
        if getattr(self, "handle", None):
            load().tina_server_destroy(self.handle)
            self.handle = None
            self._lent.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream(self, channels: int, taps: int, sample_type: str = "c64", window: str = "hann") -> int:
        sid = ctypes.c_int32()
        check(load().tina_server_stream_create(self.handle, int(channels), int(taps), SAMPLE[sample_type],
                                               WINDOW[window], ctypes.byref(sid)))
        self._streams[sid.value] = (int(channels), sample_type)
        return sid.value

    def out_rows(self, sid: int) -> int:
        P, st = self._streams[sid]
        return P if st == "c64" else P // 2 + 1

    def submit(self, sid: int, x, out) -> int:
        """Queue x (float32 or complex64) for stream sid; the output rows go to
        out (complex64, frames x channels).  Host numpy arrays are copied in and
        out by the server; CUDA tensors (both) are used in place on the device
        (TINA_REQ_DEVICE_BUFFERS).  Both are held until the request is collected."""
        if sid not in self._streams:
            raise ValueError(f"unknown stream id {sid}")
        P, st = self._streams[sid]
        r = _Request()
        r.stream_id = int(sid)
        if hasattr(x, "is_cuda"):
            import torch
            check_device_tensor(x, "input", torch.complex64 if st == "c64" else torch.float32, 1, self.device)
            check_device_tensor(out, "out", torch.complex64, 2, self.device, cols=self.out_rows(sid))
            r.flags = 1
            r.host_in = x.data_ptr() if x.numel() else None
            r.n_samples = x.numel()
            r.host_out = out.data_ptr() if out.numel() else None
            # the server waits for the work enqueued so far on the current stream (it may write x)
            r.ready_stream = torch.cuda.current_stream(self.device).cuda_stream
        else:
            check_host_array(x, "input", np.complex64 if st == "c64" else np.float32, 1)
            check_host_array(out, "out", np.complex64, 2, cols=self.out_rows(sid))
            r.host_in = x.ctypes.data if x.size else None
            r.n_samples = x.size
            r.host_out = out.ctypes.data if out.size else None
        r.out_capacity_frames = out.shape[0]
        rid = ctypes.c_uint64()
        check(load().tina_pfb_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        self._lent[rid.value] = (x, out)
        return rid.value

    @staticmethod
    def _res(r: _Result):
        return {"status": r.status, "frames": r.frames, "t_submit_us": r.t_submit_us, "t_admit_us": r.t_admit_us,
                "t_first_step_us": r.t_first_step_us, "t_done_us": r.t_done_us, "steps": r.steps}

    def poll(self, rid: int):
        r = _Result()
        st = load().tina_pfb_poll(self.handle, ctypes.c_uint64(rid), ctypes.byref(r))
        if st == 6:
            return None
        check(st)
        self._lent.pop(rid, None)
        return self._res(r)

    def submit_ptr(self, sid: int, in_ptr: int, n_samples: int, out_ptr: int, out_frames: int, device: bool,
                   ready_stream: int = 0) -> int:
        """submit() without the array checks, for a caller that owns and has
        checked its buffers (a load generator): raw pointers (device pointers
        when device is set, then ready_stream is the stream writing the input),
        the input's sample count and the output's capacity in frames.  The
        caller keeps both buffers alive until the request is collected."""
        r = _Request()
        r.stream_id = int(sid)
        r.flags = 1 if device else 0
        r.host_in = in_ptr or None
        r.n_samples = int(n_samples)
        r.host_out = out_ptr or None
        r.out_capacity_frames = int(out_frames)
        r.ready_stream = ready_stream or None
        rid = ctypes.c_uint64()
        check(load().tina_pfb_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        return rid.value

    def wait(self, rid: int, timeout_s: float = -1.0):
        r = _Result()
        us = -1 if timeout_s < 0 else int(timeout_s * 1e6)
        check(load().tina_pfb_wait(self.handle, ctypes.c_uint64(rid), us, ctypes.byref(r)))
        self._lent.pop(rid, None)
        return self._res(r)

    def cancel(self, rid: int) -> bool:
        st = load().tina_pfb_cancel(self.handle, ctypes.c_uint64(rid))
        if st == 6:
            return False
        check(st)
        return True

    def stats(self):
        s = _ServerStats()
        check(load().tina_server_get_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}


def unfold(x, width: int, stride: int = 1, out=None, stream=None):
    """Sliding-window unfold Y[i][j] = x[i*stride + j] of a 1-D float32 device
    tensor; returns the rows x width tensor."""
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise ValueError("x must be a CUDA tensor")
    check_device_tensor(x, "x", torch.float32, 1, x.device.index)
    n = x.numel()
    rows = 0 if n < width else (n - width) // stride + 1
    if out is None:
        out = torch.empty((rows, width), dtype=torch.float32, device=x.device)
    check_device_tensor(out, "out", torch.float32, 2, x.device.index, cols=int(width))
    got = ctypes.c_int64()
    check(load().tina_unfold(ctypes.c_void_p(x.data_ptr() if n else 0), n, int(width), int(stride),
                             ctypes.c_void_p(out.data_ptr() if out.numel() else 0), out.shape[0] if out.dim() == 2 else 0,
                             ctypes.byref(got), _stream_handle(stream)))
    return out[: got.value]


class Fir:
    """FIR filter y[i] = sum_k a[k] x[i-k] with arbitrary taps (host doubles)."""

    def __init__(self, taps, sample_type: str = "r32", device: int = 0):
        a = np.ascontiguousarray(taps, dtype=np.float64)
        h = ctypes.c_void_p()
        check(load().tina_fir_create(int(device), a.ctypes.data_as(ctypes.c_void_p), a.size, SAMPLE[sample_type],
                                     ctypes.byref(h)))
        self.handle = h
        self.device = int(device)
        self.complex_input = sample_type == "c64"

    def close(self):
        if getattr(self, "handle", None):
            load().tina_fir_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __call__(self, x, out=None, stream=None):
        import torch
        want = torch.complex64 if self.complex_input else torch.float32
        check_device_tensor(x, "x", want, 1, self.device)
        if out is None:
            out = torch.empty_like(x)
        check_device_tensor(out, "out", want, 1, self.device)
        if out.numel() < x.numel():
            raise ValueError(f"out holds {out.numel()} samples, fewer than the input's {x.numel()}")
        check(load().tina_fir_execute(self.handle, ctypes.c_void_p(x.data_ptr() if x.numel() else 0), x.numel(),
                                      ctypes.c_void_p(out.data_ptr() if out.numel() else 0), _stream_handle(stream)))
        return out


def schedule_simulate(ops, max_active=4, max_queued=64, frames_per_step=16, arena_bytes=1 << 30, capacity=4096):
    """Run the server's scheduler on the host (tina_server_schedule_simulate).
    ops: (kind, arg, value) tuples, kind a key of SCHED.  Returns the events
    as dicts {kind, status, id, a, b}."""
    arr = (_SchedOp * max(1, len(ops)))()
    for i, (k, arg, val) in enumerate(ops):
        arr[i].kind, arr[i].arg, arr[i].value = SCHED[k], int(arg), int(val)
    ev = (_SchedEvent * capacity)()
    n = ctypes.c_int32()
    check(load().tina_server_schedule_simulate(int(max_active), int(max_queued), int(frames_per_step),
                                               int(arena_bytes), arr, len(ops), ev, capacity, ctypes.byref(n)))
    return [{"kind": SCHED_NAME[ev[i].kind], "status": ev[i].status, "id": ev[i].id, "a": ev[i].a, "b": ev[i].b}
            for i in range(n.value)]
