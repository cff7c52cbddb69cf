"""ctypes binding of the C-ABI in ``include/lofp.h``.

Argument marshalling only: every step of the computation runs in the HIP
library ``_lib/liblofp.so``.  PyTorch is used for device buffers and streams
(``amplitudes_device`` takes CUDA/HIP tensors).  If the library has not been
built, :func:`load` raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblofp.so")

OK, EINVAL, ENOMEM, ENOTSUP, EDEVICE = 0, 1, 2, 3, 4
METHOD_AUTO, METHOD_PATHSUM, METHOD_CONTRACT = 0, 1, 2
PREC_FP64, PREC_FP32 = 0, 1
SPLIT_AUTO, SPLIT_NEVER, SPLIT_ALWAYS = 0, 1, 2

EXPORTED = (
    "lofp_last_error", "lofp_version", "lofp_circuit_create", "lofp_circuit_destroy", "lofp_light_cone",
    "lofp_bounds", "lofp_bounds_batch", "lofp_bs_table", "lofp_amplitudes_device", "lofp_amplitudes", "lofp_amplitude",
    "lofp_path_counts", "lofp_amplitudes_multi", "lofp_server_create", "lofp_server_submit",
    "lofp_server_result", "lofp_server_get_stats", "lofp_server_destroy", "lofp_amplitudes_device_noalloc",
    "lofp_all_outputs", "lofp_circuit_compiled", "lofp_graph_create", "lofp_graph_launch", "lofp_graph_destroy",
)


class LofpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lofp status {status}: {msg}")
        self.status = status


class BS(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("b", ctypes.c_int32), ("theta", ctypes.c_double), ("phi", ctypes.c_double)]


class C128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32), ("fwd_layer", ctypes.c_int32),
                ("bwd_layer", ctypes.c_int32), ("record_timing", ctypes.c_int32),
                ("frontier_budget_kb", ctypes.c_int32), ("count_work", ctypes.c_int32), ("state_limit", ctypes.c_int32),
                ("fp32_rtol", ctypes.c_double), ("autotune", ctypes.c_int32), ("split", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("fwd_layer", ctypes.c_int32), ("bwd_layer", ctypes.c_int32),
                ("dfs_levels", ctypes.c_int32), ("frontier_states", ctypes.c_int64),
                ("backward_states", ctypes.c_int64), ("bfs_states", ctypes.c_int64),
                ("dfs_leaves", ctypes.c_int64), ("dfs_edges", ctypes.c_int64), ("transitions", ctypes.c_int64),
                ("ms_plan", ctypes.c_double), ("ms_forward", ctypes.c_double), ("ms_backward", ctypes.c_double),
                ("ms_dfs", ctypes.c_double), ("ms_reduce", ctypes.c_double), ("ms_contract", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("method_used", ctypes.c_int32),
                ("split_top_keys", ctypes.c_int32), ("split_bottom_keys", ctypes.c_int32),
                ("max_state", ctypes.c_int32), ("split_cut", ctypes.c_int32), ("lds_kb", ctypes.c_int32),
                ("tuned", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("reserved")}


class Request(ctypes.Structure):
    _fields_ = [("circuit", ctypes.c_void_p), ("S", ctypes.POINTER(ctypes.c_int32)),
                ("T", ctypes.POINTER(ctypes.c_int32))]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("streams", ctypes.c_int32), ("memory_budget", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32), ("fp32_rtol", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("mean_batch", ctypes.c_double), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("fp64_fallbacks", ctypes.c_int64), ("pathsum_fallbacks", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2510_26408_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.lofp_last_error.restype = ctypes.c_char_p
    lib.lofp_version.restype = ctypes.c_char_p
    lib.lofp_circuit_create.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, ctypes.POINTER(BS),
                                        ctypes.POINTER(vp)]
    lib.lofp_circuit_destroy.argtypes = [vp]
    lib.lofp_light_cone.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, i32p, i32p, i32p, i32p]
    lib.lofp_bounds.argtypes = [vp, i32p, i32p, i32p, i32p, i32p]
    lib.lofp_bounds_batch.argtypes = [vp, i32p, ctypes.c_int32, i32p, i32p, i32p, i32p]
    lib.lofp_bs_table.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(C128)]
    lib.lofp_amplitudes_device.argtypes = [vp, i32p, ctypes.c_int32, vp, vp, ctypes.POINTER(Opts), vp,
                                           ctypes.POINTER(Stats)]
    lib.lofp_amplitudes.argtypes = [vp, i32p, ctypes.c_int32, i32p, ctypes.POINTER(C128), ctypes.POINTER(Opts),
                                    ctypes.POINTER(Stats)]
    lib.lofp_amplitude.argtypes = [vp, i32p, i32p, ctypes.POINTER(C128)]
    lib.lofp_path_counts.argtypes = [vp, i32p, ctypes.c_int32, i32p, ctypes.POINTER(ctypes.c_double)]
    lib.lofp_amplitudes_multi.argtypes = [ctypes.c_int32, ctypes.POINTER(Request), ctypes.POINTER(C128),
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Opts), vp,
                                          ctypes.POINTER(Stats)]
    lib.lofp_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.lofp_server_submit.argtypes = [vp, vp, i32p, i32p, ctypes.POINTER(ctypes.c_uint64)]
    lib.lofp_server_result.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(C128),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.lofp_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.lofp_server_destroy.argtypes = [vp]
    lib.lofp_amplitudes_device_noalloc.argtypes = [vp, i32p, ctypes.c_int32, vp, vp, ctypes.POINTER(Opts), vp]
    lib.lofp_all_outputs.argtypes = [vp, i32p, ctypes.c_int64, i32p, ctypes.POINTER(C128),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Opts)]
    lib.lofp_circuit_compiled.argtypes = [vp, i32p, i32p, ctypes.POINTER(BS), ctypes.c_int32]
    lib.lofp_graph_create.argtypes = [vp, i32p, ctypes.c_int32, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    lib.lofp_graph_launch.argtypes = [vp, vp]
    lib.lofp_graph_destroy.argtypes = [vp]
    for f in EXPORTED[2:]:
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise LofpError(rc, load().lofp_last_error().decode())


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def make_opts(method: int = METHOD_AUTO, precision: int = PREC_FP64, fwd_layer: int = -1, bwd_layer: int = -1,
              record_timing: bool = False, frontier_budget_kb: int = 0, count_work: bool = False,
              fp32_rtol: float = 0.0, state_limit: int = 0, autotune: bool = False, split: int = 0) -> Opts:
    o = Opts()
    o.method, o.precision, o.fwd_layer, o.bwd_layer = method, precision, fwd_layer, bwd_layer
    o.record_timing = 1 if record_timing else 0
    o.frontier_budget_kb = frontier_budget_kb
    o.count_work = 1 if count_work else 0
    o.fp32_rtol = fp32_rtol
    o.state_limit = state_limit
    o.autotune = 1 if autotune else 0
    o.split = split
    return o


class Circuit:
    """A circuit handle: ``layers`` is a list of layers, each a list of
    ``(a, b, theta, phi)`` with a < b (mode a = upper port; distant pairs are
    compiled to adjacent ones by the library)."""

    def __init__(self, m: int, layers: Sequence[Sequence[Tuple[int, int, float, float]]]):
        lib = load()
        self.m = int(m)
        self.depth = len(layers)
        flat = [bs for layer in layers for bs in layer]
        lens = _i32([len(l) for l in layers]) if layers else _i32([0])
        arr = (BS * max(1, len(flat)))()
        for i, (a, b, th, ph) in enumerate(flat):
            arr[i] = BS(int(a), int(b), float(th), float(ph))
        h = ctypes.c_void_p()
        _check(lib.lofp_circuit_create(self.m, len(layers), _ip(lens), arr, ctypes.byref(h)))
        self._h = h
        self.n_bs = len(flat)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lofp_circuit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- host-only queries
    def light_cone(self, layer: int, mode: int) -> Tuple[Tuple[int, int], Tuple[int, int]]:
        v = [ctypes.c_int32() for _ in range(4)]
        _check(load().lofp_light_cone(self._h, layer, mode, *[ctypes.byref(x) for x in v]))
        return (v[0].value, v[1].value), (v[2].value, v[3].value)

    def bounds(self, S, T) -> Tuple[np.ndarray, np.ndarray, bool]:
        S, T = _i32(S), _i32(T)
        lo = np.zeros((self.depth + 1) * (self.m - 1), dtype=np.int32)
        hi = np.zeros_like(lo)
        f = ctypes.c_int32()
        _check(load().lofp_bounds(self._h, _ip(S), _ip(T), _ip(lo), _ip(hi), ctypes.byref(f)))
        return lo.reshape(self.depth + 1, self.m - 1), hi.reshape(self.depth + 1, self.m - 1), bool(f.value)

    # -- device calls
    def bounds_batch(self, S, Ts) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """Device planner's bounds for every row of Ts: lo, hi [B, D+1, m-1], feasible [B]."""
        S, Ts = _i32(S), _i32(np.atleast_2d(Ts))
        B = Ts.shape[0]
        lo = np.zeros((B, self.depth + 1, self.m - 1), dtype=np.int32)
        hi = np.zeros_like(lo)
        f = np.zeros(B, dtype=np.int32)
        _check(load().lofp_bounds_batch(self._h, _ip(S), B, _ip(Ts), _ip(lo), _ip(hi), _ip(f)))
        return lo, hi, f.astype(bool)

    def bs_table(self, gate: int, N: int) -> np.ndarray:
        """Sector N of beam splitter `gate`: W[x1, y1] = <y1,N-y1|BS|x1,N-x1>."""
        out = (C128 * ((N + 1) * (N + 1)))()
        _check(load().lofp_bs_table(self._h, gate, N, out))
        a = np.frombuffer(out, dtype=np.complex128).copy()
        return a.reshape(N + 1, N + 1)

    def amplitudes(self, S, Ts, opts: Optional[Opts] = None, stats: Optional[Stats] = None) -> np.ndarray:
        S = _i32(S)
        Ts = _i32(Ts).reshape(-1, self.m)
        B = Ts.shape[0]
        out = (C128 * max(1, B))()
        _check(load().lofp_amplitudes(self._h, _ip(S), B, _ip(Ts), out,
                                      ctypes.byref(opts) if opts is not None else None,
                                      ctypes.byref(stats) if stats is not None else None))
        return np.frombuffer(out, dtype=np.complex128)[:B].copy()

    def amplitudes_device(self, S, T_dev, out_dev, opts: Optional[Opts] = None, stream=None,
                          stats: Optional[Stats] = None) -> None:
        """T_dev: int32 device tensor [B, m]; out_dev: complex128 device tensor
        [B].  ``stream``: a torch.cuda.Stream (default: the current stream)."""
        import torch

        S = _i32(S)
        assert T_dev.dtype == torch.int32 and T_dev.is_contiguous() and T_dev.shape[-1] == self.m
        assert out_dev.dtype == torch.complex128 and out_dev.is_contiguous()
        B = int(T_dev.shape[0])
        assert out_dev.numel() >= B
        if stream is None:
            stream = torch.cuda.current_stream(T_dev.device)
        _check(load().lofp_amplitudes_device(self._h, _ip(S), B, ctypes.c_void_p(T_dev.data_ptr()),
                                             ctypes.c_void_p(out_dev.data_ptr()),
                                             ctypes.byref(opts) if opts is not None else None,
                                             ctypes.c_void_p(stream.cuda_stream),
                                             ctypes.byref(stats) if stats is not None else None))

    def amplitudes_device_noalloc(self, S, T_dev, out_dev, opts: Optional[Opts] = None, stream=None) -> None:
        """The allocation-free form of :meth:`amplitudes_device` (contraction
        per pattern, per-call buffers in the library's fixed device scratch).
        The circuit must have been set up by an earlier contraction call."""
        import torch

        S = _i32(S)
        assert T_dev.dtype == torch.int32 and T_dev.is_contiguous() and T_dev.shape[-1] == self.m
        assert out_dev.dtype == torch.complex128 and out_dev.is_contiguous()
        B = int(T_dev.shape[0])
        assert out_dev.numel() >= B
        if stream is None:
            stream = torch.cuda.current_stream(T_dev.device)
        _check(load().lofp_amplitudes_device_noalloc(self._h, _ip(S), B, ctypes.c_void_p(T_dev.data_ptr()),
                                                     ctypes.c_void_p(out_dev.data_ptr()),
                                                     ctypes.byref(opts) if opts is not None else None,
                                                     ctypes.c_void_p(stream.cuda_stream)))

    def all_outputs(self, S, opts: Optional[Opts] = None) -> Tuple[np.ndarray, np.ndarray]:
        """Every output pattern of sum(S) photons (decreasing lexicographic
        order) and its amplitude: (T [count, m] int32, amp [count] complex128)."""
        S = _i32(S)
        lib = load()
        cnt = ctypes.c_int64()
        _check(lib.lofp_all_outputs(self._h, _ip(S), 0, None, None, ctypes.byref(cnt), None))
        Ts = np.zeros((cnt.value, self.m), dtype=np.int32)
        amps = (C128 * max(1, cnt.value))()
        _check(lib.lofp_all_outputs(self._h, _ip(S), cnt.value, _ip(Ts), amps, ctypes.byref(cnt),
                                    ctypes.byref(opts) if opts is not None else None))
        return Ts, np.frombuffer(amps, dtype=np.complex128)[:cnt.value].copy()

    def compiled_layers(self) -> List[List[Tuple[int, int, float, float]]]:
        """The adjacent-pair layers the library evaluates (host only)."""
        lib = load()
        nl = ctypes.c_int32()
        _check(lib.lofp_circuit_compiled(self._h, ctypes.byref(nl), None, None, 0))
        lens = np.zeros(max(1, nl.value), dtype=np.int32)
        cap = 32 * max(1, nl.value)
        arr = (BS * cap)()
        _check(lib.lofp_circuit_compiled(self._h, ctypes.byref(nl), _ip(lens), arr, cap))
        out, k = [], 0
        for l in range(nl.value):
            out.append([(arr[k + i].a, arr[k + i].b, arr[k + i].theta, arr[k + i].phi) for i in range(lens[l])])
            k += lens[l]
        return out

    def amplitude(self, S, T) -> complex:
        S, T = _i32(S), _i32(T)
        out = C128()
        _check(load().lofp_amplitude(self._h, _ip(S), _ip(T), ctypes.byref(out)))
        return complex(out.re, out.im)

    def path_counts(self, S, Ts) -> np.ndarray:
        S = _i32(S)
        Ts = _i32(Ts).reshape(-1, self.m)
        out = np.zeros(Ts.shape[0], dtype=np.float64)
        _check(load().lofp_path_counts(self._h, _ip(S), Ts.shape[0], _ip(Ts),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out


class Graph:
    """One amplitude call captured as a HIP graph: ``launch()`` re-evaluates
    the patterns now in ``T_dev`` into ``out_dev`` (both kept alive here)."""

    def __init__(self, circuit: "Circuit", S, T_dev, out_dev, opts: Optional[Opts] = None):
        import torch

        assert T_dev.dtype == torch.int32 and T_dev.is_contiguous() and T_dev.shape[-1] == circuit.m
        assert out_dev.dtype == torch.complex128 and out_dev.is_contiguous()
        self._keep = (circuit, T_dev, out_dev)
        S = _i32(S)
        h = ctypes.c_void_p()
        _check(load().lofp_graph_create(circuit.handle, _ip(S), int(T_dev.shape[0]), ctypes.c_void_p(T_dev.data_ptr()),
                                        ctypes.c_void_p(out_dev.data_ptr()),
                                        ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(self._keep[1].device)
        _check(load().lofp_graph_launch(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lofp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def amplitudes_multi(items, opts: Optional[Opts] = None, stats: Optional[Stats] = None, bounds: bool = False):
    """items: list of (Circuit, S, T).  All evaluated in one multi-circuit
    launch.  bounds=True also returns each result's rounding bound (FP32
    form; NaN for FP64)."""
    keep = []
    reqs = (Request * max(1, len(items)))()
    for i, (c, S, T) in enumerate(items):
        S, T = _i32(S), _i32(T)
        keep.append((S, T))
        reqs[i] = Request(c.handle, _ip(S), _ip(T))
    out = (C128 * max(1, len(items)))()
    eb = (ctypes.c_double * max(1, len(items)))()
    _check(load().lofp_amplitudes_multi(len(items), reqs, out, eb, ctypes.byref(opts) if opts is not None else None,
                                        None, ctypes.byref(stats) if stats is not None else None))
    amps = np.frombuffer(out, dtype=np.complex128)[:len(items)].copy()
    if bounds:
        return amps, np.frombuffer(eb, dtype=np.float64)[:len(items)].copy()
    return amps


class Server:
    """Continuous-batching request loop (native worker thread)."""

    def __init__(self, max_batch: int = 256, streams: int = 2, memory_budget: int = 1 << 30,
                 precision: int = PREC_FP64, fp32_rtol: float = 0.0):
        o = ServerOpts()
        o.max_batch, o.streams, o.memory_budget, o.precision = max_batch, streams, memory_budget, precision
        o.fp32_rtol = fp32_rtol
        h = ctypes.c_void_p()
        _check(load().lofp_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, circuit: "Circuit", S, T) -> int:
        S, T = _i32(S), _i32(T)
        t = ctypes.c_uint64()
        _check(load().lofp_server_submit(self._h, circuit.handle, _ip(S), _ip(T), ctypes.byref(t)))
        self._keep[t.value] = circuit
        return t.value

    def result(self, ticket: int, wait: bool = True):
        """(amplitude, latency_ms, err_bound) or None if not finished
        (wait=False); err_bound is NaN for the FP64 form."""
        out = C128()
        lat = ctypes.c_double()
        eb = ctypes.c_double()
        done = ctypes.c_int32()
        try:
            _check(load().lofp_server_result(self._h, ticket, 1 if wait else 0, ctypes.byref(out), ctypes.byref(lat),
                                             ctypes.byref(eb), ctypes.byref(done)))
        except LofpError:
            self._keep.pop(ticket, None)
            raise
        if not done.value:
            return None
        self._keep.pop(ticket, None)
        return complex(out.re, out.im), lat.value, eb.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().lofp_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lofp_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return load().lofp_version().decode()
