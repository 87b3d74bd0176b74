"""Python binding of libhytm.so (hybrid transfer management graph traversal, MI355X).

Argument marshalling only: every step of a run executes inside libhytm.so (HIP kernels
for gfx950 plus its host runtime).  The C ABI is declared in include/hytm.h.  PyTorch,
when present, only supplies the HIP stream a run is ordered after.

Loading fails loudly when the library has not been built (``build()``); there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhytm.so")

OK, E_INVAL, E_RANGE, E_NOMEM, E_BUDGET, E_DEVICE, E_STATE, E_UNSUPPORTED = range(8)
STATUS_NAMES = ["OK", "E_INVAL", "E_RANGE", "E_NOMEM", "E_BUDGET", "E_DEVICE", "E_STATE", "E_UNSUPPORTED"]
ALGOS = {"bfs": 0, "sssp": 1, "cc": 2, "pagerank": 3, "pr": 3, "ppr": 4, "pagerank_delta": 5, "dpr": 5}
FLOAT_ALGOS = (3, 4, 5)
MODES = {"hybrid": 0, "filter": 1, "compact": 2, "zerocopy": 3}
P_NONE, P_RESIDENT, P_FILTER, P_ZEROCOPY, P_COMPACT = range(5)
ENGINE_NAMES = ["none", "resident", "filter", "zerocopy", "compact"]
GRAPH_SYMMETRIC = 1 << 1
GRAPH_SKIP_COL_CHECK = 1 << 2
GRAPH_HUB_SORT = 1 << 3
GRAPH_NO_PACK = 1 << 4
GRAPH_WIDE_WEIGHTS = 1 << 5
UNCAPPED = (1 << 64) - 1
UNREACHED = 0xFFFFFFFF
STATIC_SELECT_MAX_PARTS = 1 << 18  # hytm_select_engines_static's limit


class HytmError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("mode", ctypes.c_int), ("partition_edges", ctypes.c_uint32),
        ("combine_k", ctypes.c_uint32), ("alpha_num", ctypes.c_uint32), ("alpha_den", ctypes.c_uint32),
        ("beta_num", ctypes.c_uint32), ("beta_den", ctypes.c_uint32), ("gamma_num", ctypes.c_uint32),
        ("gamma_den", ctypes.c_uint32), ("line_bytes", ctypes.c_uint32), ("max_outstanding", ctypes.c_uint32),
        ("index_bytes", ctypes.c_uint32), ("pr_iterations", ctypes.c_uint32), ("pr_damping", ctypes.c_double),
        ("streams", ctypes.c_uint32), ("gather_threads", ctypes.c_uint32),
        ("compact_chunk_edges", ctypes.c_uint64), ("filter_engine", ctypes.c_uint32),
        ("ppr_iterations", ctypes.c_uint32), ("reprocess", ctypes.c_uint32),
        ("dpr_max_iterations", ctypes.c_uint32), ("dpr_epsilon", ctypes.c_double),
        ("compact_gather_num", ctypes.c_uint32), ("compact_gather_den", ctypes.c_uint32),
        ("rq_distinct_lines", ctypes.c_uint32), ("zc_tie", ctypes.c_uint32), ("pr_blocking", ctypes.c_uint32),
        ("pr_block_pairs", ctypes.c_uint64), ("sssp_delta", ctypes.c_uint32),
    ]


FILTER_ENGINES = {"stream": 0, "copy": 1}


class IterStats(ctypes.Structure):
    _fields_ = [
        ("parts", ctypes.c_uint32 * 5), ("filter_tasks", ctypes.c_uint32), ("active_vertices", ctypes.c_uint64),
        ("active_edges", ctypes.c_uint64), ("bytes_filter", ctypes.c_uint64), ("bytes_compact", ctypes.c_uint64),
        ("zc_lines", ctypes.c_uint64), ("ms", ctypes.c_double),
    ]


class RunStats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("iterations", ctypes.c_uint32), ("npart", ctypes.c_uint32),
        ("nres", ctypes.c_uint32), ("part_iters", ctypes.c_uint64 * 5), ("active_vertices", ctypes.c_uint64),
        ("active_edges", ctypes.c_uint64), ("bytes_filter", ctypes.c_uint64), ("bytes_compact", ctypes.c_uint64),
        ("zc_lines", ctypes.c_uint64), ("bytes_zerocopy", ctypes.c_uint64), ("bytes_d2h", ctypes.c_uint64),
        ("bytes_resident_fill", ctypes.c_uint64), ("filter_tasks", ctypes.c_uint64),
        ("compact_chunks", ctypes.c_uint64), ("ms_total", ctypes.c_double), ("ms_fill", ctypes.c_double),
        ("ms_select", ctypes.c_double), ("iters", ctypes.POINTER(IterStats)), ("iters_cap", ctypes.c_uint32),
        ("iters_written", ctypes.c_uint32), ("mode_trace", ctypes.POINTER(ctypes.c_uint8)),
        ("mode_trace_cap", ctypes.c_uint64), ("time_kernels", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
        ("kernel_ms", ctypes.c_double * 9), ("kernel_launches", ctypes.c_uint64 * 9),
        ("kernel_items", ctypes.c_uint64 * 9), ("residual", ctypes.c_double),
        ("zc_lines_distinct", ctypes.c_uint64),
    ]


KERNEL_CLASSES = ["stats", "scan", "lists", "push_resident", "push_filter", "push_zerocopy", "push_compact",
                  "other", "pr_blocking"]


class LinkProbe(ctypes.Structure):
    _fields_ = [("h2d_copy_gbps", ctypes.c_double), ("d2h_copy_gbps", ctypes.c_double),
                ("zc_read_gbps", ctypes.c_double * 4), ("hbm_copy_gbps", ctypes.c_double),
                ("host_gather_gbps", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("lanes", ctypes.c_uint32 * 3), ("state_budget", ctypes.c_uint64),
                ("max_pending", ctypes.c_uint64)]


class QueryResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_uint32), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("m", ctypes.c_uint64), ("npart", ctypes.c_uint32),
                ("max_partition_edges", ctypes.c_uint32), ("hip_device", ctypes.c_int), ("flags", ctypes.c_uint32),
                ("hubs", ctypes.c_uint64), ("packed_weights", ctypes.c_uint32), ("weight_bytes", ctypes.c_uint32)]


# every exported entry point of include/hytm.h with its ctypes signature
_SIGNATURES = {
    "hytm_default_params": (None, [ctypes.POINTER(Params)]),
    "hytm_graph_create": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "hytm_set_device_budget": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "hytm_graph_set_parts": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]),
    "hytm_hub_order": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "hytm_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params)]),
    "hytm_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params)]),
    "hytm_graph_info_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(GraphInfo)]),
    "hytm_staging_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    "hytm_partition_bounds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]),
    "hytm_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(RunStats), ctypes.c_void_p]),
    "hytm_run_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(RunStats), ctypes.c_void_p]),
    "hytm_select_engines": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_void_p]),
    "hytm_select_engines_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "hytm_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "hytm_last_error": (ctypes.c_char_p, []),
    "hytm_link_probe": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(LinkProbe)]),
    "hytm_host_alloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]),
    "hytm_host_free": (ctypes.c_int, [ctypes.c_void_p]),
    "hytm_server_state_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32,
                                               ctypes.POINTER(ctypes.c_uint64)]),
    "hytm_server_open": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerConfig),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "hytm_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "hytm_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double,
                                        ctypes.POINTER(QueryResult)]),
    "hytm_server_close": (ctypes.c_int, [ctypes.c_void_p]),
}


class _PinnedBlock:
    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        try:
            load().hytm_host_free(self.ptr)
        except Exception:
            pass


def pinned_empty(shape, dtype=np.uint32, device: int = 0) -> np.ndarray:
    """numpy array over pinned host memory (freed with the array); pass it as `out=` so a
    run's results arrive by direct DMA."""
    dtype = np.dtype(dtype)
    count = int(np.prod(shape)) if np.ndim(shape) else int(shape)
    p = ctypes.c_void_p()
    _check(load().hytm_host_alloc(device, max(count * dtype.itemsize, 1), ctypes.byref(p)))
    block = _PinnedBlock(p)
    buf = (ctypes.c_char * max(count * dtype.itemsize, 1)).from_address(p.value)
    arr = np.frombuffer(buf, dtype=dtype, count=count).reshape(shape)
    arr.flags.writeable = True
    # keep the allocation alive as long as the array (numpy keeps `buf` via .base)
    buf._hytm_block = block
    return arr


def link_probe(bytes_: int = 1 << 30, device: int = 0) -> dict:
    """Pinned H2D/D2H copy, zero-copy read (32/64/128 B of every line, and streaming) and
    HBM copy throughput in GB/s."""
    r = LinkProbe()
    _check(load().hytm_link_probe(device, int(bytes_), ctypes.byref(r)))
    return {"h2d_copy_gbps": r.h2d_copy_gbps, "d2h_copy_gbps": r.d2h_copy_gbps,
            "zc_read_gbps": {"32B": r.zc_read_gbps[0], "64B": r.zc_read_gbps[1], "128B": r.zc_read_gbps[2],
                             "stream": r.zc_read_gbps[3]},
            "hbm_copy_gbps": r.hbm_copy_gbps, "host_gather_gbps": r.host_gather_gbps}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile libhytm.so for gfx950 with hipcc (always recompiles)."""
    from . import _build as _b
    return _b.build(verbose=verbose)


def load() -> ctypes.CDLL:
    """Load the built library; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2208_14935_amd.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise HytmError(status, load().hytm_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def hub_order(off, col):
    """Hub sorting's vertex order as the library computes it on the host: (order, hubs)
    with order[i] = original id of new vertex i and the first `hubs` entries the hubs."""
    off = np.ascontiguousarray(off)
    if off.dtype not in (np.uint32, np.uint64):
        off = off.astype(np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    n = len(off) - 1
    order = np.empty(max(n, 1), dtype=np.uint32)
    k = ctypes.c_uint64(0)
    _check(load().hytm_hub_order(n, len(col), _ptr(off), off.dtype.itemsize, _ptr(col) if len(col) else None,
                                 _ptr(order), ctypes.byref(k)))
    return order[:n], int(k.value)


def default_params() -> Params:
    p = Params()
    load().hytm_default_params(ctypes.byref(p))
    return p


def _current_stream():
    """HIP stream of PyTorch's current stream on the current device, or None."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


@dataclass
class RunResult:
    values: np.ndarray          # uint32 levels / distances / labels, or float32 ranks
    iterations: int
    stats: dict = field(default_factory=dict)
    iters: list = field(default_factory=list)
    mode_trace: np.ndarray | None = None  # iterations x npart engine codes


class Graph:
    """A CSR graph whose edge arrays live in pinned host memory (libhytm handle)."""

    def __init__(self, off, col, weights=None, symmetric: bool = False, device: int = 0,
                 check_col: bool = True, hub_sort: bool = False, pack: bool = True, narrow: bool = True):
        lib = load()
        off = np.ascontiguousarray(off)
        if off.dtype not in (np.uint32, np.uint64):
            off = off.astype(np.uint64)
        col = np.ascontiguousarray(col, dtype=np.uint32)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint32)
        if w is not None and w.shape != col.shape:
            raise ValueError("weights and col differ in length")
        self.n = len(off) - 1
        self.m = len(col)
        flags = ((GRAPH_SYMMETRIC if symmetric else 0) | (0 if check_col else GRAPH_SKIP_COL_CHECK)
                 | (GRAPH_HUB_SORT if hub_sort else 0) | (0 if pack else GRAPH_NO_PACK)
                 | (0 if narrow else GRAPH_WIDE_WEIGHTS))
        h = ctypes.c_void_p()
        self._keep = [np.zeros(1, np.uint32)]  # stand-in buffer for empty arrays
        colp = _ptr(col) if self.m else _ptr(self._keep[0])
        wp = None if w is None else (_ptr(w) if self.m else _ptr(self._keep[0]))
        _check(lib.hytm_graph_create(self.n, self.m, _ptr(off), off.dtype.itemsize, colp, wp, flags, device,
                                     ctypes.byref(h)))
        self._h = h
        self.weighted = w is not None
        self.symmetric = symmetric

    def close(self):
        srv = getattr(self, "_server", None)
        if srv is not None:
            srv.close()
        if getattr(self, "_h", None):
            load().hytm_graph_destroy(self._h)
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

    def set_parts(self, vertex_bounds):
        """Declare the graph a disjoint union of graphs with these vertex bounds (count + 1
        entries, 0 .. n); PageRank then normalizes per graph.  None undoes it."""
        if vertex_bounds is None:
            _check(load().hytm_graph_set_parts(self._h, 0, None))
            return
        b = np.ascontiguousarray(vertex_bounds, dtype=np.uint64)
        _check(load().hytm_graph_set_parts(self._h, len(b) - 1, _ptr(b)))

    def set_budget(self, edge_bytes):
        """Device bytes for edge data (None = uncapped, every partition resident)."""
        _check(load().hytm_set_device_budget(self._h, UNCAPPED if edge_bytes is None else int(edge_bytes)))

    def params(self) -> Params:
        p = Params()
        _check(load().hytm_get_params(self._h, ctypes.byref(p)))
        return p

    def set_params(self, **kw):
        """Update tunables by name (see hytm_params); mode may be given as a string."""
        p = self.params()
        for k, v in kw.items():
            if k == "mode" and isinstance(v, str):
                v = MODES[v]
            if k == "filter_engine" and isinstance(v, str):
                v = FILTER_ENGINES[v]
            if k == "compact_gather":
                p.compact_gather_num, p.compact_gather_den = int(v[0]), int(v[1])
                continue
            if k in ("alpha", "beta", "gamma"):
                setattr(p, k + "_num", int(v[0]))
                setattr(p, k + "_den", int(v[1]))
                continue
            if not hasattr(p, k):
                raise AttributeError(f"unknown parameter {k}")
            setattr(p, k, v)
        _check(load().hytm_set_params(self._h, ctypes.byref(p)))

    def reset_params(self):
        _check(load().hytm_set_params(self._h, None))

    def info(self) -> dict:
        i = GraphInfo()
        _check(load().hytm_graph_info_get(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in GraphInfo._fields_}

    def staging_bytes(self, algo: str) -> int:
        b = ctypes.c_uint64(0)
        _check(load().hytm_staging_bytes(self._h, ALGOS[algo], ctypes.byref(b)))
        return int(b.value)

    def edge_arrays(self, algo: str) -> int:
        """4-byte words the graph holds per edge for `algo`: 2 for SSSP unless its weights are
        packed into the neighbour words, else 1."""
        return 2 if ALGOS[algo] == 1 and not self.info()["packed_weights"] else 1

    def edge_bytes(self, algo: str) -> int:
        """Bytes the graph holds per edge for `algo` (d1): 4 per neighbour word, plus the weight
        kept apart for SSSP (4 bytes, or 1 with byte weights)."""
        return 4 + (self.info()["weight_bytes"] if ALGOS[algo] == 1 else 0)

    def set_resident_fraction(self, algo: str, frac: float):
        """Budget = the engines' staging + `frac` of the edge bytes `algo` reads."""
        self.set_budget(self.staging_bytes(algo) + int(frac * 4 * self.edge_arrays(algo) * self.m))

    def partition_bounds(self) -> np.ndarray:
        npart = self.info()["npart"]
        b = np.empty(npart + 1, dtype=np.uint64)
        _check(load().hytm_partition_bounds(self._h, _ptr(b), len(b)))
        return b

    def run(self, algo: str, source: int = 0, stats: bool = False, trace: bool = False, stream=None,
            out: np.ndarray | None = None, time_kernels: bool = False) -> RunResult:
        lib = load()
        a = ALGOS[algo]
        dtype = np.float32 if a in FLOAT_ALGOS else np.uint32
        if out is not None:
            if out.dtype != dtype or not out.flags.c_contiguous or out.size < self.n:
                raise ValueError(f"out must be a C-contiguous {np.dtype(dtype).name} array of n elements")
            vals = out.reshape(-1)[: self.n]
        else:
            vals = np.empty(max(self.n, 1), dtype=dtype)[: self.n]
        it = ctypes.c_uint32(0)
        st = None
        iters_buf = trace_buf = None
        if stats or trace or time_kernels:
            st = RunStats()
            st.struct_size = ctypes.sizeof(RunStats)
            st.time_kernels = 1 if time_kernels else 0
            cap = 4096
            iters_buf = (IterStats * cap)()
            st.iters = ctypes.cast(iters_buf, ctypes.POINTER(IterStats))
            st.iters_cap = cap
            if trace:
                npart = self.info()["npart"]
                trace_buf = np.zeros(npart * cap if npart * cap < (1 << 28) else npart * 64, dtype=np.uint8)
                st.mode_trace = trace_buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
                st.mode_trace_cap = len(trace_buf)
        s = stream if stream is not None else _current_stream()
        _check(lib.hytm_run(self._h, a, int(source), _ptr(vals), ctypes.byref(it),
                            ctypes.byref(st) if st is not None else None, s))
        res = RunResult(vals, int(it.value))
        if st is not None:
            arrays = ("part_iters", "kernel_ms", "kernel_launches", "kernel_items")
            res.stats = {k: (list(getattr(st, k)) if k in arrays else getattr(st, k))
                         for k, _ in RunStats._fields_
                         if k not in ("iters", "mode_trace", "struct_size", "reserved0", "time_kernels")}
            for t in range(st.iters_written):
                r = iters_buf[t]
                res.iters.append({k: (list(getattr(r, k)) if k == "parts" else getattr(r, k))
                                  for k, _ in IterStats._fields_})
            if trace:
                npart = st.npart
                rows = min(res.iterations, len(trace_buf) // max(npart, 1))
                res.mode_trace = trace_buf[: rows * npart].reshape(rows, npart).copy()
        return res

    def run_batch(self, algo: str, sources, stats: bool = False, stream=None, time_kernels: bool = False,
                  out: np.ndarray | None = None):
        """Batched BFS/SSSP/PPR from up to 64 sources in one traversal.  Returns
        (values[nsources, n] uint32 (float32 for PPR), iterations[nsources], stats dict).
        `out`, if given, is a C-contiguous array of that dtype with at least nsources*n
        elements (e.g. from pinned_empty)."""
        srcs = np.ascontiguousarray(sources, dtype=np.uint32)
        dtype = np.float32 if ALGOS[algo] in FLOAT_ALGOS else np.uint32
        if out is not None:
            if out.dtype != dtype or not out.flags.c_contiguous or out.size < len(srcs) * self.n:
                raise ValueError(f"out must be a C-contiguous {np.dtype(dtype).name} array of nsources*n elements")
            vals = out.reshape(-1)[: len(srcs) * self.n].reshape(len(srcs), self.n)
        else:
            vals = np.empty((max(len(srcs), 1), max(self.n, 1)), dtype=dtype)[: len(srcs), : self.n]
        its = np.zeros(max(len(srcs), 1), dtype=np.uint32)
        st = None
        if stats or time_kernels:
            st = RunStats()
            st.struct_size = ctypes.sizeof(RunStats)
            st.time_kernels = 1 if time_kernels else 0
        s = stream if stream is not None else _current_stream()
        _check(load().hytm_run_batch(self._h, ALGOS[algo], _ptr(srcs), len(srcs), _ptr(vals), _ptr(its),
                                     ctypes.byref(st) if st is not None else None, s))
        sd = {}
        if st is not None:
            arrays = ("part_iters", "kernel_ms", "kernel_launches", "kernel_items")
            sd = {k: (list(getattr(st, k)) if k in arrays else getattr(st, k)) for k, _ in RunStats._fields_
                  if k not in ("iters", "mode_trace", "struct_size", "reserved0", "time_kernels")}
        return vals, its[: len(srcs)], sd

    def select_engines(self, E, nA, Ea, Rq, nres: int = 0, edge_arrays: int = 1) -> np.ndarray:
        arrs = [np.ascontiguousarray(x, dtype=np.uint64) for x in (E, nA, Ea, Rq)]
        npart = len(arrs[0])
        p = np.zeros(max(npart, 1), dtype=np.uint8)
        _check(load().hytm_select_engines(self._h, npart, *(_ptr(x) for x in arrs), int(nres), int(edge_arrays),
                                          _ptr(p)))
        return p[:npart]

    def select_engines_static(self, E, nA, Ea, Rq, nres: int = 0, edge_arrays: int = 1, stream=None) -> np.ndarray:
        """select_engines through the library's static device scratch (no device
        allocation; at most STATIC_SELECT_MAX_PARTS partitions)."""
        arrs = [np.ascontiguousarray(x, dtype=np.uint64) for x in (E, nA, Ea, Rq)]
        npart = len(arrs[0])
        p = np.zeros(max(npart, 1), dtype=np.uint8)
        _check(load().hytm_select_engines_static(self._h, npart, *(_ptr(x) for x in arrs), int(nres),
                                                 int(edge_arrays), _ptr(p),
                                                 stream if stream is not None else _current_stream()))
        return p[:npart]


@dataclass
class Query:
    ticket: int
    algo: str
    source: int
    values: np.ndarray
    result: dict | None = None


class Server:
    """Query server over a Graph (hytm_server_*): BFS, SSSP and PPR queries join free lanes
    of their algorithm's lane group between iterations and leave when their traversal
    ends.  submit() returns a Query whose `values` array is filled once wait() returns."""

    def __init__(self, graph: Graph, bfs: int = 64, sssp: int = 64, ppr: int = 64, state_budget: int = 0,
                 max_pending: int = 0, pinned: bool = True):
        cfg = ServerConfig()
        cfg.struct_size = ctypes.sizeof(ServerConfig)
        cfg.lanes[0], cfg.lanes[1], cfg.lanes[2] = int(bfs), int(sssp), int(ppr)
        cfg.state_budget = int(state_budget)
        cfg.max_pending = int(max_pending)
        h = ctypes.c_void_p()
        _check(load().hytm_server_open(graph._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.graph = graph
        self.pinned = pinned
        self._live = {}
        graph._server = self

    @staticmethod
    def state_bytes(graph: Graph, algo: str, lanes: int) -> int:
        b = ctypes.c_uint64(0)
        _check(load().hytm_server_state_bytes(graph._h, ALGOS[algo], int(lanes), ctypes.byref(b)))
        return int(b.value)

    def submit(self, algo: str, source: int, out: np.ndarray | None = None) -> Query:
        n = self.graph.n
        dtype = np.float32 if ALGOS[algo] in FLOAT_ALGOS else np.uint32
        if out is None:
            out = pinned_empty(max(n, 1), dtype)[:n] if self.pinned else np.empty(max(n, 1), dtype)[:n]
        elif out.dtype != dtype or not out.flags.c_contiguous or out.size < n:
            raise ValueError(f"out must be a C-contiguous {np.dtype(dtype).name} array of n elements")
        t = ctypes.c_uint64(0)
        _check(load().hytm_server_submit(self._h, ALGOS[algo], int(source), _ptr(out), ctypes.byref(t)))
        q = Query(int(t.value), algo, int(source), out.reshape(-1)[:n])
        self._live[q.ticket] = q  # the buffer must outlive the query
        return q

    def wait(self, q: Query, timeout_ms: float = -1.0) -> Query:
        r = QueryResult()
        st = load().hytm_server_wait(self._h, q.ticket, float(timeout_ms), ctypes.byref(r))
        if st == E_STATE and q.ticket in self._live and timeout_ms >= 0:
            _check(st)  # timed out: the ticket stays live
        self._live.pop(q.ticket, None)
        q.result = {"status": r.status, "iterations": r.iterations, "queue_ms": r.queue_ms, "run_ms": r.run_ms,
                    "total_ms": r.total_ms}
        _check(st)
        return q

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            st = load().hytm_server_close(h)
            self.graph._server = None
            self._live.clear()
            _check(st)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
