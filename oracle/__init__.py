"""CPU oracle -- test infrastructure only.

Thin ctypes wrapper over ``oracle.c`` (plain single-threaded C).  Only the tests, the
smoke check and the benchmark's CPU-baseline leg import this package; the GPU library
never does.  See the header of ``oracle.c`` for what each function follows in the paper
(HyTGraph, arXiv 2208.14935).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

UNREACHED = 0xFFFFFFFF
NONE, RESIDENT, FILTER, ZEROCOPY, COMPACT = 0, 1, 2, 3, 4


def build() -> str:
    """Compile oracle.c into liboracle.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


class _CostParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in (
        "line_bytes", "max_outstanding", "d1", "d2", "alpha_num", "alpha_den",
        "beta_num", "beta_den", "gamma_num", "gamma_den", "gather_num", "gather_den", "zc_tie")]


@dataclass
class CostParams:
    """Constants of Sec. 5.1: m = 128 B, MR = 256, alpha = 0.8, beta = 0.4, gamma = 0.625.
    d1 = bytes per edge over the edge arrays read, d2 = bytes per index entry."""
    line_bytes: int = 128
    max_outstanding: int = 256
    d1: int = 4
    d2: int = 4
    alpha: tuple = (4, 5)
    beta: tuple = (2, 5)
    gamma: tuple = (5, 8)
    gather: tuple = (0, 1)  # link rate / host gather rate; (0, 1) = the paper's transfer-only Tec
    zc_tie: int = 0  # 1: a Tiz = Tef tie goes to zero-copy instead of filter

    def _c(self):
        return _CostParams(self.line_bytes, self.max_outstanding, self.d1, self.d2,
                           self.alpha[0], self.alpha[1], self.beta[0], self.beta[1],
                           self.gamma[0], self.gamma[1], self.gather[0], self.gather[1], self.zc_tie)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, u64, u32, i32, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
    sig = {
        "orc_bfs": (u32, [u64, vp, vp, u32, vp]),
        "orc_sssp": (i32, [u64, vp, vp, vp, u32, vp]),
        "orc_sssp_check": (i32, [u64, vp, vp, vp, u32, vp, vp]),
        "orc_sync_rounds": (u32, [u64, vp, vp, vp, i32, u32]),
        "orc_cc": (u64, [u64, vp, vp, vp]),
        "orc_pagerank": (None, [u64, vp, vp, dbl, u32, vp]),
        "orc_ppr": (None, [u64, vp, vp, u32, dbl, u32, vp]),
        "orc_hub_order": (u64, [u64, vp, vp, u32, u32, vp]),
        "orc_partition": (u64, [u64, vp, u64, vp]),
        "orc_partition_stats": (None, [u64, vp, vp, vp, u32, u32, vp, vp, vp]),
        "orc_partition_lines_distinct": (None, [u64, vp, vp, vp, u32, u32, vp]),
        "orc_select": (None, [u64, vp, vp, vp, vp, u64, ctypes.POINTER(_CostParams), i32, vp]),
        "orc_combine": (u64, [u64, vp, vp, u32, u64, vp, vp]),
        "orc_gather": (None, [u64, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(_EMPTY.ctypes.data)


_EMPTY = np.zeros(1, dtype=np.uint64)


def _csr(off, col):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    return off, col, len(off) - 1


def bfs(off, col, source: int):
    """(level[n] uint32, iterations) -- fewest hops from source; UNREACHED if none."""
    off, col, n = _csr(off, col)
    lvl = np.empty(max(n, 1), dtype=np.uint32)[:n]
    it = _load().orc_bfs(n, _p(off), _p(col), int(source), _p(lvl))
    return lvl, int(it)


def sssp(off, col, w, source: int):
    """dist[n] uint32 by Dijkstra; raises OverflowError if a distance reaches 2^32-1."""
    off, col, n = _csr(off, col)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    dist = np.empty(max(n, 1), dtype=np.uint32)[:n]
    if _load().orc_sssp(n, _p(off), _p(col), _p(w), int(source), _p(dist)):
        raise OverflowError("shortest distance does not fit below 2^32-1")
    return dist


def sssp_check(off, col, w, source: int, dist) -> tuple[int, int]:
    """Shortest-path certificate of `dist` (see orc_sssp_check): (0, 0) when it holds, else
    (condition 1/2/3, vertex)."""
    off, col, n = _csr(off, col)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    dist = np.ascontiguousarray(dist, dtype=np.uint32)
    if len(dist) != n or len(w) != len(col):
        raise ValueError("dist must have n entries and w one per edge")
    bad = ctypes.c_uint64(0)
    code = _load().orc_sssp_check(n, _p(off), _p(col), _p(w), int(source), _p(dist), ctypes.byref(bad))
    return int(code), int(bad.value)


def sync_rounds(off, col, w=None, kind: str = "sssp", source: int = 0) -> int:
    """Non-empty frontiers of a fully synchronous push iteration (upper bound for the
    iteration count of a run whose updates inside one iteration may be fresher)."""
    off, col, n = _csr(off, col)
    wp = _p(np.ascontiguousarray(w, dtype=np.uint32)) if w is not None else None
    return int(_load().orc_sync_rounds(n, _p(off), _p(col), wp, 0 if kind == "sssp" else 1, int(source)))


def cc(off, col):
    """(label[n] uint32 = min vertex id of the component, number of components)."""
    off, col, n = _csr(off, col)
    lab = np.empty(max(n, 1), dtype=np.uint32)[:n]
    k = _load().orc_cc(n, _p(off), _p(col), _p(lab))
    return lab, int(k)


def pagerank(off, col, d: float = 0.85, T: int = 20):
    """FP64 x_T of the synchronous power iteration (dangling mass leaks)."""
    off, col, n = _csr(off, col)
    x = np.empty(max(n, 1), dtype=np.float64)[:n]
    _load().orc_pagerank(n, _p(off), _p(col), float(d), int(T), _p(x))
    return x


def ppr(off, col, source: int, d: float = 0.85, T: int = 10):
    """FP64 personalized PageRank x_T from `source` (x_0 = e_s, restart 1 - d at s,
    dangling mass leaks)."""
    off, col, n = _csr(off, col)
    if not 0 <= source < n:
        raise ValueError("source out of range")
    x = np.empty(max(n, 1), dtype=np.float64)[:n]
    _load().orc_ppr(n, _p(off), _p(col), int(source), float(d), int(T), _p(x))
    return x


def hub_order(off, col, num: int = 8, den: int = 100):
    """Hub sorting's new vertex order: (order, k) with order[i] = original id of new vertex
    i and the first k entries the hubs."""
    off, col, n = _csr(off, col)
    order = np.empty(max(n, 1), dtype=np.uint32)[:n]
    k = _load().orc_hub_order(n, _p(off), _p(col), int(num), int(den), _p(order))
    return order, int(k)


def partition(off, target_edges: int):
    """Partition start vertices plus a final n (length npart + 1)."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    n = len(off) - 1
    bounds = np.empty(n + 2, dtype=np.uint64)
    k = _load().orc_partition(n, _p(off), int(target_edges), _p(bounds))
    return bounds[: k + 1] if n else np.zeros(1, dtype=np.uint64)


def partition_stats(bounds, off, active, arrays: int = 1, line_bytes: int = 128, distinct: bool = False,
                    weight_bytes: int | None = None):
    """(nA, Ea, Rq) per partition for the boolean frontier `active`; with distinct, Rq counts
    the different lines the active lists touch instead of Eq. 3's per-vertex requests.
    Rq covers the neighbour array (4-byte entries) and, when a weight array is read beside it
    (arrays = 2), that array too: weight_bytes bytes per entry (default 4; 1 for byte weights)."""
    wb = (4 if arrays == 2 else 0) if weight_bytes is None else int(weight_bytes)
    if (arrays == 2) != (wb > 0) or wb not in (0, 1, 4):
        raise ValueError("weight_bytes must be 1 or 4 with two arrays and 0 with one")
    bounds = np.ascontiguousarray(bounds, dtype=np.uint64)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    act = np.ascontiguousarray(active, dtype=np.uint8)
    npart = len(bounds) - 1
    nA, Ea, Rq = (np.zeros(max(npart, 1), dtype=np.uint64)[:npart] for _ in range(3))
    _load().orc_partition_stats(npart, _p(bounds), _p(off), _p(act), wb, int(line_bytes), _p(nA), _p(Ea), _p(Rq))
    if distinct:
        _load().orc_partition_lines_distinct(npart, _p(bounds), _p(off), _p(act), wb, int(line_bytes), _p(Rq))
    return nA, Ea, Rq


def select(E, nA, Ea, Rq, nres: int = 0, params: CostParams | None = None, force: int = 0):
    """Engine code per partition (NONE/RESIDENT/FILTER/ZEROCOPY/COMPACT)."""
    cp = (params or CostParams())._c()
    arrs = [np.ascontiguousarray(a, dtype=np.uint64) for a in (E, nA, Ea, Rq)]
    npart = len(arrs[0])
    p = np.zeros(max(npart, 1), dtype=np.uint8)[:npart]
    _load().orc_select(npart, *(_p(a) for a in arrs), int(nres), ctypes.byref(cp), int(force), _p(p))
    return p


def combine(p, E, k: int = 4, max_edges: int = 0):
    """List of (first, last) partition ranges, one per filter task."""
    p = np.ascontiguousarray(p, dtype=np.uint8)
    E = np.ascontiguousarray(E, dtype=np.uint64)
    npart = len(p)
    first = np.zeros(max(npart, 1), dtype=np.uint64)
    last = np.zeros(max(npart, 1), dtype=np.uint64)
    t = _load().orc_combine(npart, _p(p), _p(E), int(k), int(max_edges), _p(first), _p(last))
    return [(int(first[i]), int(last[i])) for i in range(t)]


def gather(vc, off, col):
    """(packed neighbour lists in vc order, new offsets of length len(vc)+1)."""
    vc = np.ascontiguousarray(vc, dtype=np.uint32)
    off, col, n = _csr(off, col)
    deg = (off[1:] - off[:-1])[vc] if len(vc) else np.zeros(0, np.uint64)
    packed = np.empty(max(int(deg.sum()), 1), dtype=np.uint32)[: int(deg.sum())]
    newoff = np.empty(len(vc) + 1, dtype=np.uint64)
    _load().orc_gather(len(vc), _p(vc), _p(off), _p(col), _p(packed), _p(newoff))
    return packed, newoff
