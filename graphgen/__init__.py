"""Seeded synthetic data graphs and query patterns.

Shared by the oracle's tests and by the GPU library's tests and benchmark; it
contains no part of the enumeration method.  Graphs come back as a clean CSR
(int64 row_ptr, int32 col; sorted, symmetric, no self-loops or duplicates) in
numpy arrays.  The paper's datasets (Section 7.1, Table 3) are not available;
the generators below produce graphs of the same shape classes instead.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, -O2, pthreads)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_int]
        lib.gg_chung_lu.restype = vp
        lib.gg_chung_lu.argtypes = [i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_uint64, ctypes.c_int]
        lib.gg_gnp.restype = vp
        lib.gg_gnp.argtypes = [i64, ctypes.c_double, ctypes.c_uint64]
        lib.gg_from_pairs.restype = vp
        lib.gg_from_pairs.argtypes = [i64, i64, vp, vp, ctypes.c_uint64, ctypes.c_int]
        lib.gg_n.restype = i64
        lib.gg_n.argtypes = [vp]
        lib.gg_nnz.restype = i64
        lib.gg_nnz.argtypes = [vp]
        lib.gg_copy.restype = None
        lib.gg_copy.argtypes = [vp, vp, vp]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [vp]
        lib.gg_philox4x32_10.restype = None
        lib.gg_philox4x32_10.argtypes = [vp, vp, vp]
        _lib = lib
        return lib


class CSR:
    """A clean undirected CSR graph held in numpy arrays (original vertex IDs)."""

    def __init__(self, row_ptr: np.ndarray, col: np.ndarray, name: str = ""):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.name = name

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def __repr__(self) -> str:
        return "CSR(%s n=%d m=%d)" % (self.name, self.n, self.m)


def _take(ptr, name) -> CSR:
    lib = _load()
    if not ptr:
        raise ValueError("graph generator rejected its arguments")
    try:
        n = lib.gg_n(ptr)
        nnz = lib.gg_nnz(ptr)
        rp = np.empty(n + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        lib.gg_copy(ptr, rp.ctypes.data, col.ctypes.data)
        return CSR(rp, col[:nnz], name)
    finally:
        lib.gg_free(ptr)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 2, threads: int = 0) -> CSR:
    """R-MAT graph: edge_factor * 2**scale samples, no noise, permuted IDs,
    symmetrised, self-loops dropped, deduplicated."""
    lib = _load()
    ns = int(edge_factor) << int(scale)
    return _take(lib.gg_rmat(int(scale), ns, a, b, c, int(seed), int(threads)),
                 "rmat%d_ef%d_s%d" % (scale, edge_factor, seed))


def chung_lu(n: int, dbar: float, gamma: float, seed: int, exact: bool = False, wcap: float = 0.0,
             threads: int = 0) -> CSR:
    """Chung-Lu graph with power-law weights w_i = c (i+1)^(-1/(gamma-1)),
    capped at sqrt(n * dbar) unless wcap > 0, mean weight dbar."""
    lib = _load()
    return _take(lib.gg_chung_lu(int(n), float(dbar), float(gamma), float(wcap), 1 if exact else 0,
                                 int(seed), int(threads)),
                 "chunglu_n%d_d%g_g%g_s%d" % (n, dbar, gamma, seed))


def gnp(n: int, p: float, seed: int) -> CSR:
    lib = _load()
    return _take(lib.gg_gnp(int(n), float(p), int(seed)), "gnp_n%d_p%g_s%d" % (n, p, seed))


def from_edges(n: int, edges, permute: bool = False, seed: int = 0, name: str = "") -> CSR:
    """Clean CSR from an undirected edge list (duplicates and self-loops dropped)."""
    lib = _load()
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    pu = np.ascontiguousarray(e[:, 0])
    pv = np.ascontiguousarray(e[:, 1])
    ptr = lib.gg_from_pairs(int(n), int(e.shape[0]), pu.ctypes.data, pv.ctypes.data, int(seed),
                            1 if permute else 0)
    return _take(ptr, name or "edges_n%d" % n)


class DiCSR(CSR):
    """A directed graph: its undirected skeleton (row_ptr, col: every adjacent pair,
    both ways) and its out-lists (out_rp, out_col), original IDs, lists ascending."""

    def __init__(self, row_ptr, col, out_rp, out_col, name: str = ""):
        super().__init__(row_ptr, col, name)
        self.out_rp = np.ascontiguousarray(out_rp, dtype=np.int64)
        self.out_col = np.ascontiguousarray(out_col, dtype=np.int32)

    @property
    def arcs(self) -> int:
        return int(self.out_col.shape[0])


def orient(g: CSR, p_both: float, seed: int) -> DiCSR:
    """Directions for every edge {u, v} of g: both with probability p_both, else
    one of the two, each with probability 1/2 (numpy's Philox generator, seeded).
    The skeleton of the result is g itself."""
    rng = np.random.Generator(np.random.Philox(int(seed)))
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    v = g.col.astype(np.int64)
    keep = u < v
    eu, ev = u[keep], v[keep]
    both = rng.random(eu.shape[0]) < p_both
    pick = rng.integers(0, 2, eu.shape[0])
    fwd = both | (pick == 0)
    bwd = both | (pick == 1)
    src = np.concatenate([eu[fwd], ev[bwd]])
    dst = np.concatenate([ev[fwd], eu[bwd]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    out_rp = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=g.n), out=out_rp[1:])
    return DiCSR(g.row_ptr, g.col, out_rp, dst.astype(np.int32), g.name + "_dir%g_s%d" % (p_both, seed))


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block (exposed for the generator's known-answer test)."""
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.empty(4, dtype=np.uint32)
    lib.gg_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return [int(x) for x in o]


# --------------------------------------------------------------------------
# named small graphs (closed-form test cases)
# --------------------------------------------------------------------------
def complete(n: int) -> CSR:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name="K%d" % n)


def cycle(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], name="C%d" % n)


def path(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], name="P%d" % n)


def grid(r: int, c: int) -> CSR:
    e = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                e.append((v, v + 1))
            if i + 1 < r:
                e.append((v, v + c))
    return from_edges(r * c, e, name="grid%dx%d" % (r, c))


def complete_bipartite(a: int, b: int) -> CSR:
    return from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)], name="K%d,%d" % (a, b))


def hypercube(d: int) -> CSR:
    n = 1 << d
    return from_edges(n, [(v, v ^ (1 << i)) for v in range(n) for i in range(d) if v < v ^ (1 << i)],
                      name="Q%d" % d)


def petersen() -> CSR:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return from_edges(10, outer + spokes + inner, name="petersen")


def star(leaves: int) -> CSR:
    return from_edges(leaves + 1, [(0, i + 1) for i in range(leaves)], name="S%d" % leaves)
