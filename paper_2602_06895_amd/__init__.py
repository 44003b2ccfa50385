"""Python binding of the MI355X phase-space library (libmsx.so, C ABI in
include/msx.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libmsx.so.  torch supplies device buffers and the current HIP stream.  There
is no CPU fallback: without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsx.so")

FP64, MIXED = 0, 1
META_N_CHANNELS, META_DIMS, META_N_MOMENTA, META_HADRONIC = 0, 1, 2, 3
META_VEGAS_BINS, META_MAX_MOMENTA, META_PROCESS, META_DEVICE, META_PRECISION = 4, 5, 6, 7, 8
META_EVENTS_PER_THREAD, META_GRID, META_COUNTER, META_FLOW, META_SPECIALIZED = 9, 10, 11, 12, 13
COUNTER_AUTO = 2 ** 64 - 1
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_DEVICE", 3: "ERR_OOM", 4: "ERR_UNSUPPORTED", 5: "ERR_STATE"}

EXPORTS = ["msx_last_error", "msx_create_channels", "msx_destroy", "msx_get_meta", "msx_uniform", "msx_map",
           "msx_weight", "msx_sample", "msx_stats", "msx_reset_stats", "msx_vegas_accumulate",
           "msx_vegas_update", "msx_get_grid", "msx_set_grid", "msx_unweight_eff",
           "msx_flow_last_error", "msx_flow_create", "msx_flow_destroy", "msx_flow_param_count",
           "msx_flow_set_params", "msx_flow_get_params", "msx_flow_forward", "msx_flow_inverse",
           "msx_flow_gradient", "msx_flow_train_step", "msx_flow_sample", "msx_sample_device",
           "msx_sample_graph_create", "msx_graph_launch", "msx_graph_destroy", "msx_set_launch", "msx_autotune",
           "msx_inverse_map", "msx_multichannel_density", "msx_unweight", "msx_observables", "msx_cut",
           "msx_histogram", "msx_vegas_adapt", "msx_allocate_counts",
           "msx_sample_noalloc", "msx_get_state", "msx_set_state", "msx_attach_flow", "msx_flow_get_state",
           "msx_flow_set_state", "msx_flow_dims", "msx_specialize"]
OBS_E, OBS_PT, OBS_ETA, OBS_PHI, OBS_M, OBS_PT_RANK, OBS_DR_HARDEST = range(7)
FLOW_BF16, FLOW_FP32 = 0, 1
SAMPLE_ACCUMULATE_VEGAS, SAMPLE_USE_FLOW, SAMPLE_ADVANCE_COUNTER = 1, 2, 4


class MsxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmsx.so and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build()")
    # torch first: its HIP runtime is then the one the library binds to (two
    # runtimes in one process do not share devices)
    import torch  # noqa: F401

    L = C.CDLL(path)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sigs = {
        "msx_last_error": ([vp], C.c_char_p),
        "msx_create_channels": ([C.c_char_p, i32, i32, C.POINTER(vp)], C.c_int),
        "msx_destroy": ([vp], C.c_int),
        "msx_get_meta": ([vp, i32, i32, C.POINTER(i64)], C.c_int),
        "msx_uniform": ([vp, u64, u64, u64, i64, i32, vp, vp], C.c_int),
        "msx_map": ([vp, i32, i64, vp, vp, vp, vp, vp, vp], C.c_int),
        "msx_inverse_map": ([vp, i32, i64, vp, vp, vp, vp, vp], C.c_int),
        "msx_multichannel_density": ([vp, i32, i64, vp, vp, vp, vp, vp], C.c_int),
        "msx_unweight": ([vp, vp, i64, C.c_double, C.c_uint64, C.c_uint64, C.c_uint64, vp, vp, vp, vp], C.c_int),
        "msx_observables": ([vp, i32, i64, vp, vp, i32, vp, vp], C.c_int),
        "msx_cut": ([vp, i64, vp, i32, vp, vp, vp, vp], C.c_int),
        "msx_histogram": ([vp, i64, vp, vp, i32, C.c_double, C.c_double, vp, vp], C.c_int),
        "msx_weight": ([vp, i32, i64, vp, vp, vp, vp, vp, vp], C.c_int),
        "msx_sample": ([vp, vp, u64, u64, u64, i32, vp, vp, vp, vp, vp], C.c_int),
        "msx_vegas_adapt": ([vp, i64, i32, dbl, u64, u64, u64, vp, vp], C.c_int),
        "msx_sample_noalloc": ([vp, vp, u64, u64, u64, vp, vp, vp, vp, vp], C.c_int),
        "msx_get_state": ([vp, vp, C.POINTER(C.c_size_t)], C.c_int),
        "msx_set_state": ([vp, vp, C.c_size_t], C.c_int),
        "msx_attach_flow": ([vp, i32, vp, i64, u64, C.POINTER(i32), vp], C.c_int),
        "msx_flow_get_state": ([vp, vp, C.POINTER(C.c_size_t)], C.c_int),
        "msx_flow_set_state": ([vp, vp, C.c_size_t], C.c_int),
        "msx_flow_dims": ([vp, C.POINTER(i32)], C.c_int),
        "msx_allocate_counts": ([i32, vp, i64, dbl, vp], C.c_int),
        "msx_stats": ([vp, vp, vp], C.c_int),
        "msx_reset_stats": ([vp, vp], C.c_int),
        "msx_vegas_accumulate": ([vp, i32, i64, vp, vp, vp], C.c_int),
        "msx_vegas_update": ([vp, dbl, vp], C.c_int),
        "msx_get_grid": ([vp, i32, vp], C.c_int),
        "msx_set_grid": ([vp, i32, vp], C.c_int),
        "msx_unweight_eff": ([vp, vp, i64, dbl, C.POINTER(dbl), C.POINTER(dbl), vp], C.c_int),
        "msx_sample_device": ([vp, vp, u64, u64, vp, i64, i32, vp, vp, vp, vp, vp, vp], C.c_int),
        "msx_sample_graph_create": ([vp, vp, u64, u64, vp, i64, i32, vp, vp, vp, vp, vp, C.POINTER(vp)], C.c_int),
        "msx_graph_launch": ([vp, vp], C.c_int),
        "msx_graph_destroy": ([vp], C.c_int),
        "msx_set_launch": ([vp, i32, i32], C.c_int),
        "msx_autotune": ([vp, vp, u64, i32, C.POINTER(dbl)], C.c_int),
        "msx_specialize": ([vp, i32], C.c_int),
        "msx_flow_last_error": ([vp], C.c_char_p),
        "msx_flow_create": ([i32, i32, i32, i32, i32, i32, C.POINTER(vp)], C.c_int),
        "msx_flow_destroy": ([vp], C.c_int),
        "msx_flow_param_count": ([vp, C.POINTER(i64)], C.c_int),
        "msx_flow_set_params": ([vp, vp, i64], C.c_int),
        "msx_flow_get_params": ([vp, vp, i64], C.c_int),
        "msx_flow_forward": ([vp, i64, vp, vp, vp, vp], C.c_int),
        "msx_flow_inverse": ([vp, i64, vp, vp, vp, vp], C.c_int),
        "msx_flow_gradient": ([vp, i64, vp, vp, vp, vp, vp, vp], C.c_int),
        "msx_flow_train_step": ([vp, i64, vp, vp, vp, C.c_float, vp, vp], C.c_int),
        "msx_flow_sample": ([vp, vp, i32, i64, u64, u64, u64, vp, vp, vp, vp, vp, vp, vp], C.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(t):
    """Device (or host numpy) pointer of a tensor/array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


class Context:
    """One msx context: compiled channels, VEGAS grids and statistics on one GPU.

    `desc` is a process description (dict or JSON string, see include/msx.h)."""

    def __init__(self, desc, device: int = 0, precision: int = FP64):
        import torch

        self.torch = torch
        self.L = load_library()
        text = desc if isinstance(desc, str) else json.dumps(desc)
        h = C.c_void_p()
        st = self.L.msx_create_channels(text.encode(), precision, device, C.byref(h))
        if st != 0:
            raise MsxError(st, self.L.msx_last_error(None).decode())
        self.h = h
        self.device = torch.device("cuda", device)
        self.n_channels = self._meta(META_N_CHANNELS, 0)
        self.max_momenta = self._meta(META_MAX_MOMENTA, 0)
        self.dims = [self._meta(META_DIMS, c) for c in range(self.n_channels)]
        self.n_momenta = [self._meta(META_N_MOMENTA, c) for c in range(self.n_channels)]
        self.hadronic = [bool(self._meta(META_HADRONIC, c)) for c in range(self.n_channels)]
        self.nbins = [self._meta(META_VEGAS_BINS, c) for c in range(self.n_channels)]
        self.precision = self._meta(META_PRECISION, 0)
        self._flows = {}  # attached flows, kept alive while attached

    # -- plumbing ------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise MsxError(st, self.L.msx_last_error(self.h).decode())

    def _meta(self, key, index):
        v = C.c_int64()
        self._check(self.L.msx_get_meta(self.h, key, index, C.byref(v)))
        return v.value

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _empty(self, *shape, dtype=None):
        return self.torch.empty(shape, dtype=dtype or self.torch.float64, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.L.msx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API -----------------------------------------------------------------
    def uniform(self, seed: int, stream_id: int, e0: int, n: int, d: int):
        y = self._empty(d, n)
        self._check(self.L.msx_uniform(self.h, seed, stream_id, e0, n, d, _ptr(y), self._stream()))
        return y

    def _check_channel(self, channel: int):
        if not (0 <= channel < self.n_channels):
            raise MsxError(1, f"channel index {channel} out of range")

    def _check_y(self, channel: int, y):
        self._check_channel(channel)
        if y.dim() != 2 or y.shape[0] != self.dims[channel] or y.dtype != self.torch.float64 or y.device != self.device:
            raise ValueError(f"y must be a float64 [{self.dims[channel]}][n] tensor on {self.device}")

    def map(self, channel: int, y, weight: bool = False):
        self._check_y(channel, y)
        n = y.shape[1]
        np_ = self.n_momenta[channel]
        out = {"p": self._empty(4, np_, n), "jac": self._empty(n)}
        out["x1x2"] = self._empty(2, n) if self.hadronic[channel] else None
        out["w"] = self._empty(n) if weight else None
        y = y.contiguous()
        self._check(self.L.msx_map(self.h, channel, n, _ptr(y), _ptr(out["p"]), _ptr(out["x1x2"]),
                                   _ptr(out["jac"]), _ptr(out["w"]), self._stream()))
        return out

    def inverse_map(self, channel: int, p, x1x2=None, jac: bool = True):
        """Uniforms y [d][n] that the channel maps to the lab-frame momenta p
        [4][np][n] (and x1x2 [2][n] for hadronic beams), with the forward
        Jacobian at y (the channel density is 1/jac)."""
        self._check_channel(channel)
        n = p.shape[2]
        if tuple(p.shape) != (4, self.n_momenta[channel], n) or p.dtype != self.torch.float64:
            raise ValueError(f"p must be a float64 [4][{self.n_momenta[channel]}][n] tensor")
        p = p.contiguous()
        x1x2 = x1x2.contiguous() if x1x2 is not None else None
        out = {"y": self._empty(self.dims[channel], n), "jac": self._empty(n) if jac else None}
        self._check(self.L.msx_inverse_map(self.h, channel, n, _ptr(p), _ptr(x1x2), _ptr(out["y"]),
                                           _ptr(out["jac"]), self._stream()))
        return out

    def observables(self, process: int, p, spec):
        """spec: list of (kind, particle labels, rank); returns [k][n] values."""
        rows = []
        for kind, labels, rank in spec:
            m = 0
            for q in labels:
                m |= 1 << q
            rows += [kind, m, rank, 0]
        a = np.ascontiguousarray(rows, dtype=np.int32)
        k = len(spec)
        n = p.shape[2]
        out = self._empty(k, n)
        p = p.contiguous()
        self._check(self.L.msx_observables(self.h, process, n, _ptr(p), a.ctypes.data_as(C.c_void_p), k, _ptr(out),
                                           self._stream()))
        return out

    def cut(self, x, lo, hi, w):
        """w[e] = 0 unless lo[j] <= x[j][e] < hi[j] for all j (in place)."""
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        x = x.contiguous()
        self._check(self.L.msx_cut(self.h, x.shape[1], _ptr(x), x.shape[0], lo.ctypes.data_as(C.c_void_p),
                                   hi.ctypes.data_as(C.c_void_p), _ptr(w), self._stream()))
        return w

    def histogram(self, x, w, bins: int, lo: float, hi: float):
        """[2][bins] (sum w, sum w^2) of x over equal bins of [lo, hi)."""
        out = self._empty(2, bins)
        self._check(self.L.msx_histogram(self.h, x.shape[0], _ptr(x.contiguous()), _ptr(w.contiguous()), bins,
                                         float(lo), float(hi), _ptr(out), self._stream()))
        return out

    def unweight(self, w, w_max: float, seed: int, stream_id: int = 0, counter_offset: int = 0):
        """Hit-or-miss unweighting of w [n] (device float64) against w_max:
        kept indices (increasing), their unit weights max(1, w / w_max) and
        the count (a device int64 tensor of one element)."""
        n = w.shape[0]
        w = w.contiguous()
        keep = self.torch.empty(max(n, 1), dtype=self.torch.int64, device=self.device)
        uw = self._empty(max(n, 1))
        count = self.torch.zeros(1, dtype=self.torch.int64, device=self.device)
        self._check(self.L.msx_unweight(self.h, _ptr(w), n, float(w_max), seed, stream_id, counter_offset,
                                        _ptr(keep), _ptr(uw), _ptr(count), self._stream()))
        return {"keep": keep, "uw": uw, "count": count}

    def multichannel_density(self, process: int, p, x1x2, alpha):
        """g(p) = sum_c alpha_c / J_c(y_c(p)) over the channels of `process`
        (alpha: one a-priori weight per channel of the process, host)."""
        n = p.shape[2]
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        p = p.contiguous()
        x1x2 = x1x2.contiguous() if x1x2 is not None else None
        g = self._empty(n)
        self._check(self.L.msx_multichannel_density(self.h, process, n, _ptr(p), _ptr(x1x2),
                                                    a.ctypes.data_as(C.c_void_p), _ptr(g), self._stream()))
        return g

    def weight(self, channel: int, p, x1x2, jac, alpha: bool = False):
        n = jac.shape[0]
        self._check_channel(channel)
        if tuple(p.shape) != (4, self.n_momenta[channel], n):
            raise ValueError(f"p must be [4][{self.n_momenta[channel]}][{n}]")
        w = self._empty(n)
        a = self._empty(n) if alpha else None
        self._check(self.L.msx_weight(self.h, channel, n, _ptr(p), _ptr(x1x2), _ptr(jac), _ptr(w), _ptr(a),
                                      self._stream()))
        return (w, a) if alpha else w

    def sample(self, counts, seed: int, stream_id: int = 0, counter_offset: int = 0, out: dict | None = None,
               want_chan: bool = True, flags: int = 0):
        counts = np.ascontiguousarray(counts, dtype=np.int64)
        if counts.shape != (self.n_channels,):
            raise ValueError(f"counts must have {self.n_channels} entries")
        if (counts < 0).any():
            raise MsxError(1, "negative event count")
        N = int(counts.sum())
        if out is not None and (out["p"].shape[1] != self.max_momenta or out["p"].shape[2] < N or out["w"].shape[0] < N):
            raise ValueError("output buffers are too small")
        if out is None:
            out = {"p": self._empty(4, self.max_momenta, N), "w": self._empty(N),
                   "x1x2": self._empty(2, N) if any(self.hadronic) else None,
                   "chan": self._empty(N, dtype=self.torch.int32) if want_chan else None}
        self._check(self.L.msx_sample(self.h, counts.ctypes.data, seed, stream_id, counter_offset, flags,
                                      _ptr(out["p"]), _ptr(out["x1x2"]), _ptr(out["w"]), _ptr(out.get("chan")),
                                      self._stream()))
        return out

    def sample_device(self, counts, seed: int, stream_id: int, counter_offset, out: dict, status=None,
                      flags: int = 0):
        """msx_sample_device: counts (int64 [C]) and counter_offset (uint64 [1],
        stored as int64) are device tensors; out holds buffers of one capacity."""
        cap = out["w"].shape[0]
        self._check(self.L.msx_sample_device(self.h, _ptr(counts), seed, stream_id, _ptr(counter_offset), cap,
                                             flags, _ptr(out["p"]), _ptr(out.get("x1x2")), _ptr(out["w"]),
                                             _ptr(out.get("chan")), _ptr(status), self._stream()))

    def sample_graph(self, counts, seed: int, stream_id: int, counter_offset, out: dict, status=None,
                     flags: int = 0):
        """Capture msx_sample_device into a HIP graph; returns a SampleGraph."""
        cap = out["w"].shape[0]
        g = C.c_void_p()
        self._check(self.L.msx_sample_graph_create(self.h, _ptr(counts), seed, stream_id, _ptr(counter_offset), cap,
                                                   flags, _ptr(out["p"]), _ptr(out.get("x1x2")), _ptr(out["w"]),
                                                   _ptr(out.get("chan")), _ptr(status), C.byref(g)))
        return SampleGraph(self, g, (counts, counter_offset, out, status))

    def sample_buffers(self, capacity: int, want_chan: bool = True) -> dict:
        return {"p": self._empty(4, self.max_momenta, capacity), "w": self._empty(capacity),
                "x1x2": self._empty(2, capacity) if any(self.hadronic) else None,
                "chan": self._empty(capacity, dtype=self.torch.int32) if want_chan else None}

    def set_launch(self, events_per_thread: int, grid: int = 0):
        self._check(self.L.msx_set_launch(self.h, events_per_thread, grid))

    def launch_shape(self):
        return self._meta(META_EVENTS_PER_THREAD, 0), self._meta(META_GRID, 0)

    def autotune(self, counts, seed: int = 1, reps: int = 3) -> float:
        c = np.ascontiguousarray(counts, dtype=np.int64)
        ms = C.c_double()
        self._check(self.L.msx_autotune(self.h, c.ctypes.data, seed, reps, C.byref(ms)))
        return ms.value

    def specialize(self, on: bool = True):
        """Sample launches use (on) the kernel compiled for these channels
        with their tables as constants (bit-identical results), or the
        default kernel (off)."""
        self._check(self.L.msx_specialize(self.h, 1 if on else 0))

    @property
    def specialized(self) -> bool:
        return bool(self._meta(META_SPECIALIZED, 0))

    @property
    def specialized_kernels(self) -> int:
        """Kernels the specialised sample launches (channel groups)."""
        return self._meta(META_SPECIALIZED, 0)

    def stats(self) -> np.ndarray:
        out = np.zeros((self.n_channels, 5))
        self._check(self.L.msx_stats(self.h, out.ctypes.data, self._stream()))
        return out

    def reset_stats(self):
        self._check(self.L.msx_reset_stats(self.h, self._stream()))

    def vegas_accumulate(self, channel: int, y, w):
        self._check_y(channel, y)
        if w.dim() != 1 or w.shape[0] != y.shape[1] or w.dtype != self.torch.float64:
            raise ValueError("w must be float64 [n] matching y")
        self._check(self.L.msx_vegas_accumulate(self.h, channel, w.shape[0], _ptr(y.contiguous()),
                                                _ptr(w.contiguous()), self._stream()))

    def vegas_update(self, alpha: float = 0.5):
        self._check(self.L.msx_vegas_update(self.h, alpha, self._stream()))

    def get_grid(self, channel: int) -> np.ndarray:
        out = np.zeros((self.dims[channel], self.nbins[channel] + 1))
        self._check(self.L.msx_get_grid(self.h, channel, out.ctypes.data))
        return out

    def set_grid(self, channel: int, edges):
        e = np.ascontiguousarray(edges, dtype=np.float64)
        if e.shape != (self.dims[channel], self.nbins[channel] + 1):
            raise ValueError("grid shape mismatch")
        self._check(self.L.msx_set_grid(self.h, channel, e.ctypes.data))

    def get_state(self) -> bytes:
        """msx_get_state: grids, histograms, statistics, launch shape, event
        counter and attached flows as one blob."""
        n = C.c_size_t()
        self._check(self.L.msx_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self.L.msx_get_state(self.h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, blob: bytes):
        self._check(self.L.msx_set_state(self.h, blob, len(blob)))

    def counter(self) -> int:
        return self._meta(META_COUNTER, 0) % 2 ** 64

    def attach_flow(self, channel: int, flow, n_check: int = 0, seed: int = 1):
        """msx_attach_flow: returns (enabled, (rel. variance VEGAS, flow))."""
        self._check_channel(channel)
        en = C.c_int32()
        rv = np.full(2, np.nan)
        self._check(self.L.msx_attach_flow(self.h, channel, flow.h if flow is not None else None, n_check, seed,
                                           C.byref(en), rv.ctypes.data))
        self._flows[channel] = flow
        return bool(en.value), (float(rv[0]), float(rv[1]))

    def flow_state(self, channel: int) -> int:
        return self._meta(META_FLOW, channel)

    def unweight_eff(self, w, overweight: float = 1e-3):
        if w.dtype != self.torch.float64 or w.device != self.device:
            raise ValueError("w must be a float64 tensor on the context's device")
        eff, wmax = C.c_double(), C.c_double()
        self._check(self.L.msx_unweight_eff(self.h, _ptr(w.contiguous()), w.shape[0], overweight, C.byref(eff),
                                            C.byref(wmax), self._stream()))
        return eff.value, wmax.value


class SampleGraph:
    """An instantiated HIP graph of one device-count sample launch; keeps the
    buffers it was captured with alive."""

    def __init__(self, ctx: Context, handle, buffers):
        self.ctx, self.h, self._buffers = ctx, handle, buffers

    def launch(self):
        self.ctx._check(self.ctx.L.msx_graph_launch(self.h, self.ctx._stream()))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.msx_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Flow:
    """Rational-quadratic spline coupling flow on one GPU (include/msx_flow.h).

    Event arrays are float32 [d][n] CUDA tensors; parameters are a flat float32
    vector in the layout the header documents."""

    def __init__(self, dims: int, layers: int = 8, bins: int = 16, hidden: int = 128, mlp: int = FLOW_BF16,
                 device: int = 0):
        import torch

        self.torch = torch
        self.L = load_library()
        h = C.c_void_p()
        st = self.L.msx_flow_create(dims, layers, bins, hidden, mlp, device, C.byref(h))
        if st != 0:
            raise MsxError(st, self.L.msx_flow_last_error(None).decode())
        self.h = h
        self.dims, self.layers, self.bins, self.hidden, self.mlp = dims, layers, bins, hidden, mlp
        self.device = torch.device("cuda", device)
        n = C.c_int64()
        self._check(self.L.msx_flow_param_count(self.h, C.byref(n)))
        self.n_params = n.value

    def _check(self, st):
        if st != 0:
            raise MsxError(st, self.L.msx_flow_last_error(self.h).decode())

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _events(self, t, name):
        if t.dim() != 2 or t.shape[0] != self.dims or t.dtype != self.torch.float32 or t.device != self.device:
            raise ValueError(f"{name} must be a float32 [{self.dims}][n] tensor on {self.device}")
        return t.contiguous()

    def close(self):
        if getattr(self, "h", None):
            self.L.msx_flow_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (self.n_params,):
            raise ValueError(f"expected {self.n_params} parameters")
        self._check(self.L.msx_flow_set_params(self.h, p.ctypes.data, p.shape[0]))

    def get_state(self) -> bytes:
        n = C.c_size_t()
        self._check(self.L.msx_flow_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self.L.msx_flow_get_state(self.h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, blob: bytes):
        self._check(self.L.msx_flow_set_state(self.h, blob, len(blob)))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(self.L.msx_flow_get_params(self.h, p.ctypes.data, p.shape[0]))
        return p

    def forward(self, u):
        u = self._events(u, "u")
        n = u.shape[1]
        y = self.torch.empty_like(u)
        ld = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        self._check(self.L.msx_flow_forward(self.h, n, _ptr(u), _ptr(y), _ptr(ld), self._stream()))
        return y, ld

    def inverse(self, y):
        y = self._events(y, "y")
        n = y.shape[1]
        u = self.torch.empty_like(y)
        lq = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        self._check(self.L.msx_flow_inverse(self.h, n, _ptr(y), _ptr(u), _ptr(lq), self._stream()))
        return u, lq

    def _batch(self, y, wfj, logq_old):
        y = self._events(y, "y")
        n = y.shape[1]
        if wfj.shape != (n,) or wfj.dtype != self.torch.float64 or logq_old.shape != (n,) or \
                logq_old.dtype != self.torch.float32:
            raise ValueError("wfj must be float64 [n] and logq_old float32 [n]")
        return y, wfj.contiguous(), logq_old.contiguous(), n

    def gradient(self, y, wfj, logq_old):
        y, wfj, lqo, n = self._batch(y, wfj, logq_old)
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(1, dtype=self.torch.float64, device=self.device)
        self._check(self.L.msx_flow_gradient(self.h, n, _ptr(y), _ptr(wfj), _ptr(lqo), _ptr(g), _ptr(loss),
                                             self._stream()))
        return g, loss

    def train_step(self, y, wfj, logq_old, lr: float = 1e-3):
        y, wfj, lqo, n = self._batch(y, wfj, logq_old)
        loss = self.torch.empty(1, dtype=self.torch.float64, device=self.device)
        self._check(self.L.msx_flow_train_step(self.h, n, _ptr(y), _ptr(wfj), _ptr(lqo), lr, _ptr(loss),
                                               self._stream()))
        return loss

    def sample(self, ctx: "Context", channel: int, n: int, seed: int, stream_id: int = 0, counter_offset: int = 0):
        ctx._check_channel(channel)
        t = self.torch
        np_ = ctx.n_momenta[channel]
        out = {"y": t.empty(self.dims, n, dtype=t.float32, device=self.device),
               "logq": t.empty(n, dtype=t.float32, device=self.device),
               "p": ctx._empty(4, np_, n), "x1x2": ctx._empty(2, n) if ctx.hadronic[channel] else None,
               "wfj": ctx._empty(n), "w": ctx._empty(n)}
        self._check(self.L.msx_flow_sample(self.h, ctx.h, channel, n, seed, stream_id, counter_offset,
                                           _ptr(out["y"]), _ptr(out["logq"]), _ptr(out["p"]), _ptr(out["x1x2"]),
                                           _ptr(out["wfj"]), _ptr(out["w"]), self._stream()))
        return out


def adapt_vegas(ctx: Context, n_per_channel: int, iterations: int, alpha: float = 0.5, seed: int = 1,
                stream_id: int = 1, counter_offset: int = 0):
    """msx_vegas_adapt: the library's adaptation phase (every iteration one
    fused sample of n_per_channel events per channel that accumulates the
    VEGAS histograms, then a grid refinement).  Returns the statistics [C][5]
    of the last iteration; leaves the context's statistics reset."""
    out = np.zeros((ctx.n_channels, 5))
    ctx._check(ctx.L.msx_vegas_adapt(ctx.h, n_per_channel, iterations, alpha, seed, stream_id, counter_offset,
                                     out.ctypes.data, ctx._stream()))
    return out


def neyman_counts(stats: np.ndarray, total: int, floor_frac: float = 0.01) -> np.ndarray:
    """msx_allocate_counts: events per channel proportional to each channel's
    weight standard deviation, with a floor of floor_frac * total each."""
    L = load_library()
    st = np.ascontiguousarray(stats, dtype=np.float64)
    if st.ndim != 2 or st.shape[1] != 5:
        raise ValueError("stats must be [C][5]")
    counts = np.zeros(st.shape[0], dtype=np.int64)
    rc = L.msx_allocate_counts(st.shape[0], st.ctypes.data, int(total), float(floor_frac), counts.ctypes.data)
    if rc != 0:
        raise MsxError(rc, L.msx_last_error(None).decode())
    return counts
