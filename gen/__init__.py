"""Seeded synthetic graph inputs (R-MAT, Erdos-Renyi, explicit edge lists).

Inputs only: this module builds CSR arrays (rows sorted, self-loops and duplicate edges
removed), the symmetrized CSR, per-edge weights and source vertices.  It holds no part of
the traversal or cost-model arithmetic and is shared by the CPU oracle and the GPU
library's tests and benchmark.  The C source is ``gen.c``; ``build()`` compiles it with
gcc into ``libhytmgen.so`` next to it.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libhytmgen.so")
_lib = None

# R-MAT quadrant probabilities used for every synthetic graph here
RMAT_ABC = (0.57, 0.19, 0.19)


def build() -> str:
    """Compile gen.c into libhytmgen.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fPIC", "-shared", "-pthread",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, u64, u32, i32, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
    lib.gen_rmat.restype = vp
    lib.gen_rmat.argtypes = [i32, u64, dbl, dbl, dbl, u64]
    lib.gen_er.restype = vp
    lib.gen_er.argtypes = [u64, u64, u64]
    lib.gen_from_pairs.restype = vp
    lib.gen_from_pairs.argtypes = [u64, u64, vp, vp]
    lib.gen_symmetrize_csr.restype = vp
    lib.gen_symmetrize_csr.argtypes = [u64, vp, vp]
    lib.gen_num_vertices.restype = u64
    lib.gen_num_vertices.argtypes = [vp]
    lib.gen_num_edges.restype = u64
    lib.gen_num_edges.argtypes = [vp]
    lib.gen_copy_out.restype = None
    lib.gen_copy_out.argtypes = [vp, vp, vp]
    lib.gen_free.restype = None
    lib.gen_free.argtypes = [vp]
    lib.gen_weights.restype = None
    lib.gen_weights.argtypes = [u64, vp, vp, u64, u32, vp]
    lib.gen_sources.restype = u64
    lib.gen_sources.argtypes = [u64, vp, u64, u64, vp]
    lib.gen_set_threads.restype = None
    lib.gen_set_threads.argtypes = [i32]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _take(h):
    lib = _load()
    if not h:
        raise ValueError("graph generation failed (bad parameters or out of memory)")
    try:
        n = lib.gen_num_vertices(h)
        m = lib.gen_num_edges(h)
        off = np.empty(n + 1, dtype=np.uint64)
        col = np.empty(max(m, 1), dtype=np.uint32)[:m]
        lib.gen_copy_out(h, _ptr(off), _ptr(col) if m else _ptr(np.empty(1, np.uint32)))
    finally:
        lib.gen_free(h)
    return off, col


def set_threads(t: int) -> None:
    _load().gen_set_threads(int(t))


def rmat(scale: int, edge_factor: float = 16, seed: int = 0, abc=RMAT_ABC):
    """R-MAT graph on 2**scale vertices from edge_factor * 2**scale samples."""
    a, b, c = abc
    ns = int(edge_factor * (1 << scale))
    return _take(_load().gen_rmat(int(scale), ns, a, b, c, int(seed)))


def er(n: int, m: int, seed: int = 0):
    """Erdos-Renyi G(n, m): m uniform directed samples, deduplicated."""
    return _take(_load().gen_er(int(n), int(m), int(seed)))


def from_pairs(n: int, src, dst):
    """CSR from explicit (src[i], dst[i]) pairs (deduplicated, self-loops dropped)."""
    s = np.ascontiguousarray(src, dtype=np.uint32)
    d = np.ascontiguousarray(dst, dtype=np.uint32)
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    if len(s) == 0:
        return np.zeros(int(n) + 1, dtype=np.uint64), np.zeros(0, dtype=np.uint32)
    return _take(_load().gen_from_pairs(int(n), len(s), _ptr(s), _ptr(d)))


def symmetrize(off: np.ndarray, col: np.ndarray):
    """CSR of E union reverse(E)."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    n = len(off) - 1
    c = col if len(col) else np.zeros(1, np.uint32)
    return _take(_load().gen_symmetrize_csr(n, _ptr(off), _ptr(c)))


def weights(off: np.ndarray, col: np.ndarray, seed: int, maxw: int = 64) -> np.ndarray:
    """w(u, v) = 1 + hash(u, v, seed) mod maxw, uniform in [1, maxw]."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    w = np.empty(max(len(col), 1), dtype=np.uint32)
    if len(col):
        _load().gen_weights(len(off) - 1, _ptr(off), _ptr(col), int(seed), int(maxw), _ptr(w))
    return w[: len(col)]


def disjoint_union(graphs):
    """One CSR holding graphs [(off, col[, w]), ...] side by side: graph i's vertex v
    becomes bounds[i] + v.  Returns (off, col, w or None, bounds)."""
    ns = [len(g[0]) - 1 for g in graphs]
    bounds = np.concatenate([[0], np.cumsum(ns)]).astype(np.uint64)
    ms = [len(g[1]) for g in graphs]
    ebase = np.concatenate([[0], np.cumsum(ms)]).astype(np.uint64)
    off = np.empty(int(bounds[-1]) + 1, dtype=np.uint64)
    col = np.empty(int(ebase[-1]), dtype=np.uint32)
    have_w = all(len(g) > 2 and g[2] is not None for g in graphs)
    w = np.empty(int(ebase[-1]), dtype=np.uint32) if have_w else None
    for i, g in enumerate(graphs):
        b, e = int(bounds[i]), int(ebase[i])
        off[b:b + ns[i]] = np.asarray(g[0][:-1], dtype=np.uint64) + e
        col[e:e + ms[i]] = np.asarray(g[1], dtype=np.uint32) + np.uint32(b)
        if have_w:
            w[e:e + ms[i]] = g[2]
    off[-1] = ebase[-1]
    return off, col, w, bounds


def sources(off: np.ndarray, k: int, seed: int) -> np.ndarray:
    """k distinct vertices with out-degree >= 1, uniform, from a seeded counter stream."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    out = np.empty(max(int(k), 1), dtype=np.uint32)
    got = _load().gen_sources(len(off) - 1, _ptr(off), int(k), int(seed), _ptr(out))
    return out[:got]


# ------------------------------------------------------------------ CSR cache
_CSR_MAGIC = b"HYTMCSR1"


def save_csr(path: str, off: np.ndarray, col: np.ndarray) -> None:
    """Write a CSR (uint64 offsets, uint32 neighbours) to `path` in a raw binary layout:
    8-byte magic, n and m as little-endian uint64, then off[0..n] and col[0..m).  The file
    is written under a temporary name and renamed, so a reader never sees half of it."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    n, m = len(off) - 1, len(col)
    if n < 0 or int(off[-1]) != m:
        raise ValueError("off[-1] must equal len(col)")
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "wb") as fh:
        fh.write(_CSR_MAGIC)
        fh.write(np.array([n, m], dtype="<u8").tobytes())
        off.tofile(fh)
        col.tofile(fh)
    os.replace(tmp, path)


def load_csr(path: str, mmap: bool = False):
    """(off, col) from a file written by save_csr; with mmap the arrays map the file
    read-only instead of being read into memory."""
    with open(path, "rb") as fh:
        head = fh.read(24)
    if len(head) != 24 or head[:8] != _CSR_MAGIC:
        raise ValueError(f"{path}: not a CSR cache file")
    n, m = (int(x) for x in np.frombuffer(head[8:], dtype="<u8"))
    if os.path.getsize(path) != 24 + 8 * (n + 1) + 4 * m:
        raise ValueError(f"{path}: truncated CSR cache file")
    if mmap:
        off = np.memmap(path, dtype=np.uint64, mode="r", offset=24, shape=(n + 1,))
        col = np.memmap(path, dtype=np.uint32, mode="r", offset=24 + 8 * (n + 1), shape=(m,))
    else:
        with open(path, "rb") as fh:
            fh.seek(24)
            off = np.fromfile(fh, dtype=np.uint64, count=n + 1)
            col = np.fromfile(fh, dtype=np.uint32, count=m)
    if len(off) != n + 1 or len(col) != m or int(off[-1]) != m:
        raise ValueError(f"{path}: inconsistent CSR cache file")
    return off, col


def source_tag() -> str:
    """A short hash of the generator's source: cache keys include it, so a changed generator
    never reuses a graph (or anything computed from one) made by an older version."""
    h = hashlib.sha256()
    for f in (_SRC, os.path.abspath(__file__)):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def rmat_cached(scale: int, edge_factor: float = 16, seed: int = 0, cache_dir: str | None = None):
    """rmat(scale, edge_factor, seed), read from (or written to) `cache_dir` when one is
    given (default: the HYTM_GRAPH_CACHE environment variable; none = no cache)."""
    cache_dir = cache_dir if cache_dir is not None else os.environ.get("HYTM_GRAPH_CACHE")
    if not cache_dir:
        return rmat(scale, edge_factor, seed)
    path = os.path.join(cache_dir, f"rmat{scale}-ef{edge_factor:g}-s{seed}-{source_tag()}.csr")
    if os.path.exists(path):
        return load_csr(path)
    off, col = rmat(scale, edge_factor, seed)
    os.makedirs(cache_dir, exist_ok=True)
    save_csr(path, off, col)
    return off, col
