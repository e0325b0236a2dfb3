"""ORACLE -- test infrastructure only.

Plain CPU implementations of what the GPU library computes, for the test
suite, the smoke check and the benchmark's CPU-baseline leg.  The GPU library
never imports this package, and this package never imports the library.

* ``enumerate_query`` wraps the C backtracking enumerator in huge_oracle.c
  (subgraph enumeration as defined in Section 2 of the paper; see that file's
  header for the exact result definition: count, set-hash sum and xor, and
  per-prefix level counts).
* ``brute_force`` is the definition with nothing in between, for tiny graphs:
  it tries every injective map of the query into the data graph and keeps the
  distinct image edge sets.
* ``set_hash`` is the per-subgraph hash h(g) written from its definition, used
  by ``brute_force``.
* ``mlp_ref`` (a submodule) is the FP64 reference of the learned cardinality
  model: forward pass, loss gradient and one Adam step.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "huge_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

MODE_SB = 0
MODE_CANON = 1
MODE_ALL = 2
KMAX = 8
_M64 = (1 << 64) - 1


def build(force: bool = True) -> str:
    """Compile huge_oracle.c into liboracle.so with gcc."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("hash_sum", ctypes.c_uint64), ("hash_xor", ctypes.c_uint64),
                ("level_counts", ctypes.c_uint64 * KMAX)]


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
        ci = ctypes.c_int
        lib.orc_enumerate.restype = ci
        lib.orc_enumerate.argtypes = [i64, vp, vp, ci, ci, vp, ci, vp, ci, vp, ctypes.c_uint32, ctypes.c_uint32,
                                      ci, ci, ci, ci, ci, ctypes.c_uint32, ctypes.c_uint32, vp, vp, vp, ci,
                                      ctypes.POINTER(_Result)]
        lib.orc_enumerate_directed.restype = ci
        lib.orc_enumerate_directed.argtypes = [i64, vp, vp, vp, vp, ci, ci, vp, ci, vp, ctypes.c_uint32,
                                               ctypes.c_uint32, ci, ci, vp, vp, ci, ctypes.POINTER(_Result)]
        lib.orc_automorphisms_directed.restype = ci
        lib.orc_automorphisms_directed.argtypes = [ci, ci, vp]
        lib.orc_automorphisms.restype = ci
        lib.orc_automorphisms.argtypes = [ci, ci, vp, vp, ci]
        lib.orc_sb_pairs.restype = ci
        lib.orc_sb_pairs.argtypes = [ci, ci, vp, vp]
        lib.orc_check_csr.restype = ci
        lib.orc_check_csr.argtypes = [i64, vp, vp]
        lib.orc_ranks.restype = ci
        lib.orc_ranks.argtypes = [i64, vp, vp]
        lib.orc_mix64.restype = ctypes.c_uint64
        lib.orc_mix64.argtypes = [ctypes.c_uint64]
        _lib = lib
        return lib


def _qarr(qedges):
    e = np.ascontiguousarray(np.asarray(qedges, dtype=np.int32).reshape(-1, 2))
    return e


def enumerate_query(row_ptr, col, k, qedges, mode=MODE_SB, order=None, sb_pairs=None, slice_count=1,
                    slice_id=0, threads=0, slice_vertex=0, slice_pair=None, slice_mode=0, slice2=None,
                    ranks=None, induced=False, vlabels=None, qlabels=None):
    """Run the C enumerator.  Returns a dict with count, hash_sum, hash_xor and
    level_counts (list of KMAX ints; entry d counts partial maps of the first
    d+1 vertices of the order used).  slice_pair=(a, b) slices on the ordered
    pair of images (r(f(a)), r(f(b))) instead of one vertex.  slice_mode=1
    makes vertex slices strided (rank mod S) instead of mixed, and pair slices
    strided by the pair's entry in the rank-relabelled CSR; slice2=(c, S2, s2)
    adds a second vertex slice on query vertex c, slice2=(c, d, S2, s2) a second
    pair slice on (c, d).  ranks: the output of
    ranks(row_ptr) for this graph, to skip recomputing them.  induced=True
    counts induced occurrences only (every non-edge of q maps to a non-edge).
    vlabels (one int per data vertex) and qlabels (one per query vertex, -1 =
    any) make it a labelled match: every query vertex's image carries its label."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    e = _qarr(qedges)
    o = None if order is None else np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    if sb_pairs is None:
        nsb, sbp = -1, None
    else:
        sbp = np.ascontiguousarray(np.asarray(sb_pairs, dtype=np.int32).reshape(-1, 2))
        nsb = int(sbp.shape[0])
        if nsb == 0:
            sbp = np.zeros((1, 2), dtype=np.int32)
    rk = None
    if ranks is not None:
        rk = np.ascontiguousarray(ranks, dtype=np.int32)
        if rk.shape != (rp.shape[0] - 1,):
            raise ValueError("ranks must hold one entry per vertex")
    vl = None if vlabels is None else np.ascontiguousarray(vlabels, dtype=np.int32)
    ql = None if qlabels is None else np.ascontiguousarray(qlabels, dtype=np.int32)
    if vl is not None and vl.shape != (rp.shape[0] - 1,):
        raise ValueError("vlabels must hold one entry per vertex")
    if ql is not None and ql.shape != (int(k),):
        raise ValueError("qlabels must hold one entry per query vertex")
    r = _Result()
    st = lib.orc_enumerate(int(rp.shape[0] - 1), rp.ctypes.data, cl.ctypes.data, int(k), int(e.shape[0]),
                           e.ctypes.data, int(mode) | (4 if induced else 0), None if o is None else o.ctypes.data, nsb,
                           None if sbp is None else sbp.ctypes.data, int(slice_count), int(slice_id),
                           int(slice_pair[0] if slice_pair else slice_vertex),
                           int(slice_pair[1] if slice_pair else -1), int(slice_mode),
                           int(slice2[0]) if slice2 else -1, int(slice2[1]) if slice2 and len(slice2) == 4 else -1,
                           int(slice2[-2]) if slice2 else 1, int(slice2[-1]) if slice2 else 0,
                           None if rk is None else rk.ctypes.data,
                           None if vl is None else vl.ctypes.data, None if ql is None else ql.ctypes.data,
                           int(threads), ctypes.byref(r))
    if st != 0:
        raise ValueError("oracle rejected the query or order")
    return {"count": int(r.count), "hash_sum": int(r.hash_sum), "hash_xor": int(r.hash_xor),
            "level_counts": [int(x) for x in r.level_counts]}


def enumerate_directed(row_ptr, col, out_rp, out_col, k, qedges, mode=MODE_SB, order=None, slice_count=1,
                       slice_id=0, slice_vertex=0, slice_mode=0, threads=0, vlabels=None, qlabels=None):
    """A directed query on a directed graph: row_ptr/col is the graph's undirected
    skeleton, out_rp/out_col its out-lists (original IDs, ascending), qedges the
    query's directed edges a -> b.  Matches keep every edge's direction and are
    counted once per class of the direction-keeping automorphisms; the set-hash
    hashes the image's skeleton edges."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    drp = np.ascontiguousarray(out_rp, dtype=np.int64)
    dcl = np.ascontiguousarray(out_col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    if dcl.size == 0:
        dcl = np.zeros(1, dtype=np.int32)
    e = _qarr(qedges)
    o = None if order is None else np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    vl = None if vlabels is None else np.ascontiguousarray(vlabels, dtype=np.int32)
    ql = None if qlabels is None else np.ascontiguousarray(qlabels, dtype=np.int32)
    r = _Result()
    st = lib.orc_enumerate_directed(int(rp.shape[0] - 1), rp.ctypes.data, cl.ctypes.data, drp.ctypes.data,
                                    dcl.ctypes.data, int(k), int(e.shape[0]), e.ctypes.data, int(mode),
                                    None if o is None else o.ctypes.data, int(slice_count), int(slice_id),
                                    int(slice_vertex), int(slice_mode), None if vl is None else vl.ctypes.data,
                                    None if ql is None else ql.ctypes.data, int(threads), ctypes.byref(r))
    if st != 0:
        raise ValueError("oracle rejected the query or order")
    return {"count": int(r.count), "hash_sum": int(r.hash_sum), "hash_xor": int(r.hash_xor),
            "level_counts": [int(x) for x in r.level_counts]}


def automorphisms_directed(k, qedges):
    """|Aut(q)| of a directed query: the permutations keeping every edge's direction."""
    e = _qarr(qedges)
    n = _load().orc_automorphisms_directed(int(k), int(e.shape[0]), e.ctypes.data)
    if n < 0:
        raise ValueError("malformed query")
    return n


def automorphisms(k, qedges):
    lib = _load()
    e = _qarr(qedges)
    cap = 40320
    perms = np.zeros(cap * k, dtype=np.int32)
    n = lib.orc_automorphisms(int(k), int(e.shape[0]), e.ctypes.data, perms.ctypes.data, cap)
    if n < 0:
        raise ValueError("malformed query")
    return perms[: n * k].reshape(n, k)


def sb_pairs(k, qedges):
    lib = _load()
    e = _qarr(qedges)
    out = np.zeros(56, dtype=np.int32)
    n = lib.orc_sb_pairs(int(k), int(e.shape[0]), e.ctypes.data, out.ctypes.data)
    if n < 0:
        raise ValueError("malformed query")
    return [tuple(int(x) for x in out[2 * i:2 * i + 2]) for i in range(n)]


def check_csr(row_ptr, col):
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return int(lib.orc_check_csr(int(rp.shape[0] - 1), rp.ctypes.data, cl.ctypes.data))


def ranks(row_ptr):
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    n = int(rp.shape[0] - 1)
    out = np.zeros(max(n, 1), dtype=np.int32)
    lib.orc_ranks(n, rp.ctypes.data, out.ctypes.data)
    return out[:n]


def mix64(x: int) -> int:
    return int(_load().orc_mix64(int(x) & _M64))


# --------------------------------------------------------------------------
# brute force (tiny graphs only)
# --------------------------------------------------------------------------
def _py_mix(x: int) -> int:
    # SplitMix64 finalizer (Steele, Lea, Flood 2014), arithmetic mod 2^64
    x &= _M64
    x ^= x >> 30
    x = (x * 0xBF58476D1CE4E5B9) & _M64
    x ^= x >> 27
    x = (x * 0x94D049BB133111EB) & _M64
    x ^= x >> 31
    return x


def set_hash(edge_set, rank) -> int:
    """h(g) for a subgraph given as a set of undirected data edges."""
    s = 0
    for (a, b) in edge_set:
        ra, rb = int(rank[a]), int(rank[b])
        lo, hi = min(ra, rb), max(ra, rb)
        s = (s + _py_mix((lo << 32) | hi)) & _M64
    return _py_mix(s)


def brute_force(row_ptr, col, k, qedges):
    """Definition-level enumeration for tiny graphs (n <= ~12): every injective
    map of the k query vertices into V_G that keeps every query edge is tried;
    subgraphs are the distinct image edge sets.  Returns count, hash_sum,
    hash_xor, and the number of maps (= count * |Aut(q)|)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    cl = np.asarray(col, dtype=np.int32)
    n = int(rp.shape[0] - 1)
    adj = set()
    for u in range(n):
        for e in range(int(rp[u]), int(rp[u + 1])):
            adj.add((u, int(cl[e])))
    deg = np.diff(rp)
    order = sorted(range(n), key=lambda u: (int(deg[u]), u))
    rank = [0] * n
    for i, u in enumerate(order):
        rank[u] = i
    qe = [tuple(int(x) for x in e) for e in np.asarray(qedges).reshape(-1, 2)]
    images = set()
    nmaps = 0
    for f in itertools.permutations(range(n), k):
        if all((f[a], f[b]) in adj for (a, b) in qe):
            nmaps += 1
            images.add(frozenset((min(f[a], f[b]), max(f[a], f[b])) for (a, b) in qe))
    hs, hx = 0, 0
    for g in images:
        h = set_hash(g, rank)
        hs = (hs + h) & _M64
        hx ^= h
    return {"count": len(images), "hash_sum": hs, "hash_xor": hx, "maps": nmaps}


def _iso_key(k, edges):
    """Smallest sorted edge tuple over every relabelling of vertices 0..k-1 (the
    isomorphism class of a small graph, by brute force)."""
    best = None
    for p in itertools.permutations(range(k)):
        t = tuple(sorted((min(p[a], p[b]), max(p[a], p[b])) for a, b in edges))
        if best is None or t < best:
            best = t
    return best


def iso_key(k, edges):
    """The isomorphism class key of a small graph on vertices 0..k-1 (see _iso_key)."""
    return _iso_key(k, [tuple(x) for x in edges])


def _connected(k, edges):
    adj = {v: set() for v in range(k)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    seen, stack = {0}, [0]
    while stack:
        for b in adj[stack.pop()]:
            if b not in seen:
                seen.add(b)
                stack.append(b)
    return len(seen) == k


def motif_counts(row_ptr, col, k):
    """Motif counts by the definitions (Section 2), for tiny graphs: over every
    k-vertex set X, the induced subgraph G[X] (if connected) adds one induced
    occurrence of its isomorphism class, and every connected spanning subgraph of
    G[X] adds one non-induced occurrence (a subgraph of G isomorphic to its class).
    Returns {class key: (noninduced, induced)}, keys from _iso_key."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    cl = np.asarray(col, dtype=np.int32)
    n = int(rp.shape[0] - 1)
    adj = set()
    for u in range(n):
        for e in range(int(rp[u]), int(rp[u + 1])):
            adj.add((u, int(cl[e])))
    out = {}
    for X in itertools.combinations(range(n), k):
        ind = [(a, b) for a in range(k) for b in range(a + 1, k) if (X[a], X[b]) in adj]
        if not _connected(k, ind):
            continue
        key = _iso_key(k, ind)
        nonind, induced = out.get(key, (0, 0))
        out[key] = (nonind, induced + 1)
        for r in range(k - 1, len(ind) + 1):
            for sub in itertools.combinations(ind, r):
                if _connected(k, sub):
                    sk = _iso_key(k, sub)
                    a, b = out.get(sk, (0, 0))
                    out[sk] = (a + 1, b)
    return out
