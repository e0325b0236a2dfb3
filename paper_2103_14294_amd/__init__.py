"""Python binding of libhuge.so (include/huge.h): argument marshalling only.

Every step of the enumeration runs in the library's HIP kernels; this module
only converts arguments, hands device memory and streams from PyTorch to the
library, and turns status codes into exceptions.  It refuses to run without
the built library: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhuge.so")
KMAX = 8

HUGE_OK, HUGE_STOPPED = 0, 1
STATUS = {0: "HUGE_OK", 1: "HUGE_STOPPED", -1: "HUGE_EINVAL", -2: "HUGE_ENOMEM", -3: "HUGE_EDEVICE",
          -4: "HUGE_EGRAPH", -5: "HUGE_EQUERY", -6: "HUGE_EORDER", -7: "HUGE_EOVERFLOW"}
HOST_PTRS, DEVICE_PTRS, NO_VALIDATE, NO_HUB_BITMAP = 0x1, 0x2, 0x4, 0x8
PLAN_COST_MODEL, PLAN_LEARNED, PLAN_VERIFY, PLAN_INDUCED, PLAN_ALL_MAPS = 0x0, 0x1, 0x2, 0x4, 0x8
ENGINE_AUTO, ENGINE_LEVELS, ENGINE_PERSISTENT, ENGINE_GRAPH = 0, 1, 2, 3
EXEC_NO_HASH, EXEC_SLICE2_PAIR = 0x1, 0x2
SLICE_MIX, SLICE_STRIDE = 0, 1
STRAT_BSEARCH, STRAT_WAVE_STAGED, STRAT_LANE_MERGE, STRAT_MERGE_SHORT, STRAT_MERGE_LONG = 0, 1, 2, 3, 4
STRAT_BLOCK_MERGE, STRAT_BLOCK_MERGE_LONG = 5, 6
STRAT_COUNT = 7

EXPORTED = [
    "huge_exec_opts_default", "huge_load_csr", "huge_graph_free", "huge_graph_get_info", "huge_graph_export",
    "huge_plan_create", "huge_plan_free", "huge_plan_info", "huge_workspace_size", "huge_count",
    "huge_enumerate", "huge_count_batch", "huge_last_error",
    "huge_model_create", "huge_model_free", "huge_model_set", "huge_model_get", "huge_model_forward",
    "huge_model_grad", "huge_model_train", "huge_plan_features", "huge_plan_create_learned",
    "huge_autotune", "huge_graph_digest", "huge_plan_prefix", "huge_plan_create_learned2", "huge_device_name",
    "huge_batch_workspace_size", "huge_plan_estimates", "huge_count_noalloc", "huge_noalloc_capacity",
    "huge_motif_count", "huge_load_csr_labelled", "huge_plan_create_labelled",
    "huge_plan_create_bushy", "huge_plan_bushy_nodes", "huge_count_bushy", "huge_plan_create_bushy_tree",
    "huge_segment_rows", "huge_load_csr_directed", "huge_plan_create_directed", "huge_count_paths",
]
MOTIF_KMAX, MOTIF_MAX = 6, 112
MLP_F, MLP_H = 128, 256
MLP_PARAMS = MLP_F * MLP_H + 2 * MLP_H + 1


class HugeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status
        self.name = STATUS.get(status, str(status))


class Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("hash_sum", ctypes.c_uint64), ("hash_xor", ctypes.c_uint64),
                ("level_counts", ctypes.c_uint64 * KMAX), ("query_ms", ctypes.c_double),
                ("peak_frontier_bytes", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("steals", ctypes.c_uint64), ("kernel_ms", ctypes.c_double * 4),
                ("kernel_launches", ctypes.c_uint64 * 4), ("alg_bytes", ctypes.c_double * 4),
                ("level_work", ctypes.c_uint64 * KMAX), ("workgroups", ctypes.c_uint64),
                ("wg_busy_ms_mean", ctypes.c_double), ("wg_busy_ms_std", ctypes.c_double)]

    def to_dict(self):
        return {"count": int(self.count), "hash_sum": int(self.hash_sum), "hash_xor": int(self.hash_xor),
                "level_counts": [int(x) for x in self.level_counts], "query_ms": float(self.query_ms),
                "peak_frontier_bytes": int(self.peak_frontier_bytes), "launches": int(self.launches),
                "steals": int(self.steals), "kernel_ms": [float(x) for x in self.kernel_ms],
                "kernel_launches": [int(x) for x in self.kernel_launches],
                "alg_bytes": [float(x) for x in self.alg_bytes],
                "level_work": [int(x) for x in self.level_work], "workgroups": int(self.workgroups),
                "wg_busy_ms_mean": float(self.wg_busy_ms_mean), "wg_busy_ms_std": float(self.wg_busy_ms_std)}


class Motif(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_edges", ctypes.c_int32), ("edges", ctypes.c_int32 * 30),
                ("noninduced", ctypes.c_uint64), ("induced", ctypes.c_uint64), ("hash_sum", ctypes.c_uint64),
                ("hash_xor", ctypes.c_uint64)]


class ExecOpts(ctypes.Structure):
    _fields_ = [("frontier_cap_bytes", ctypes.c_uint64), ("chunk_rows", ctypes.c_int64),
                ("strategy", ctypes.c_int32), ("engine", ctypes.c_int32), ("work_stealing", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("slice_count", ctypes.c_uint32), ("slice_id", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("profile", ctypes.c_int32), ("slice_vertex", ctypes.c_int32), ("exec_flags", ctypes.c_uint32),
                ("slice_mode", ctypes.c_uint32), ("tune", ctypes.c_void_p), ("work_limit", ctypes.c_int64),
                ("slice2_vertex", ctypes.c_int32), ("slice2_count", ctypes.c_uint32), ("slice2_id", ctypes.c_uint32),
                ("slice2_vertex2", ctypes.c_int32)]


TUNE_BUCKETS = 5


class TuneTable(ctypes.Structure):
    _fields_ = [("strategy", (ctypes.c_int32 * TUNE_BUCKETS) * (KMAX + 1)),
                ("chunk_rows", ctypes.c_int64 * (KMAX + 1)),
                ("ms", (ctypes.c_double * TUNE_BUCKETS) * (KMAX + 1)),
                ("items", (ctypes.c_int64 * TUNE_BUCKETS) * (KMAX + 1))]

    def to_dict(self):
        return {"strategy": [list(r) for r in self.strategy], "chunk_rows": list(self.chunk_rows),
                "ms": [list(r) for r in self.ms], "items": [list(r) for r in self.items]}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for j in range(KMAX + 1):
            t.chunk_rows[j] = int(d["chunk_rows"][j])
            for c in range(TUNE_BUCKETS):
                t.strategy[j][c] = int(d["strategy"][j][c])
                t.ms[j][c] = float(d["ms"][j][c])
                t.items[j][c] = int(d["items"][j][c])
        return t


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("degree_hist", ctypes.c_uint64 * 32), ("degree_moments", ctypes.c_double * 8),
                ("load_ms", ctypes.c_double), ("device_bytes", ctypes.c_uint64), ("hub_count", ctypes.c_int64),
                ("hub_min_degree", ctypes.c_int64)]


BUSHY_UNIT, BUSHY_EXTEND, BUSHY_PULL_HASH, BUSHY_PUSH = 0, 1, 2, 3
BUSHY_KINDS = {0: "unit", 1: "extend", 2: "pull_hash", 3: "push"}
BUSHY_MAX_EDGES, BUSHY_MAX_NODES = 15, 29


class BushyNode(ctypes.Structure):
    _fields_ = [("edge_mask", ctypes.c_uint32), ("vertex_mask", ctypes.c_uint32), ("kind", ctypes.c_int32),
                ("left", ctypes.c_int32), ("right", ctypes.c_int32), ("star_root", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("est_rows", ctypes.c_double), ("cost", ctypes.c_double)]


EMIT_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                           ctypes.c_int32)

_lib = None
_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load libhuge.so and declare its signatures.  Raises if it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError("libhuge.so is not built (run __graft_entry__.build() or "
                               "python paper_2103_14294_amd/build.py); there is no fallback path")
        # One HIP runtime per process: the library shares streams and device memory with
        # torch, so torch's runtime is loaded first and the library binds to it (the two
        # runtimes have one soname; whichever loads first serves both).
        try:
            _torch()
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        st = ctypes.c_int
        lib.huge_exec_opts_default.restype = st
        lib.huge_exec_opts_default.argtypes = [ctypes.POINTER(ExecOpts)]
        lib.huge_load_csr.restype = st
        lib.huge_load_csr.argtypes = [i64, i64, vp, vp, u32, vp, ctypes.POINTER(vp)]
        lib.huge_load_csr_labelled.restype = st
        lib.huge_load_csr_labelled.argtypes = [i64, i64, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]
        lib.huge_plan_create_labelled.restype = st
        lib.huge_plan_create_labelled.argtypes = [vp, i32, i32, vp, vp, vp, u32, ctypes.POINTER(vp)]
        lib.huge_graph_free.restype = None
        lib.huge_graph_free.argtypes = [vp]
        lib.huge_graph_get_info.restype = st
        lib.huge_graph_get_info.argtypes = [vp, ctypes.POINTER(GraphInfo)]
        lib.huge_graph_export.restype = st
        lib.huge_graph_export.argtypes = [vp, vp, vp, vp]
        lib.huge_plan_create.restype = st
        lib.huge_plan_create.argtypes = [vp, i32, i32, vp, vp, u32, ctypes.POINTER(vp)]
        lib.huge_plan_free.restype = None
        lib.huge_plan_free.argtypes = [vp]
        lib.huge_plan_info.restype = st
        lib.huge_plan_info.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.huge_plan_estimates.restype = st
        lib.huge_plan_estimates.argtypes = [vp, vp]
        lib.huge_motif_count.restype = st
        lib.huge_motif_count.argtypes = [vp, i32, ctypes.POINTER(ExecOpts), ctypes.POINTER(Motif),
                                         ctypes.POINTER(i32)]
        lib.huge_plan_create_bushy.restype = st
        lib.huge_plan_create_bushy.argtypes = [vp, ctypes.POINTER(GraphInfo), i32, i32, vp, vp, ctypes.c_double,
                                               ctypes.POINTER(ctypes.c_void_p)]
        lib.huge_plan_create_bushy_tree.restype = st
        lib.huge_plan_create_bushy_tree.argtypes = [vp, ctypes.POINTER(GraphInfo), i32, i32, vp, vp, vp, i32,
                                                    ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)]
        lib.huge_load_csr_directed.restype = st
        lib.huge_load_csr_directed.argtypes = [i64, i64, vp, vp, ctypes.c_uint32, vp, ctypes.POINTER(ctypes.c_void_p)]
        lib.huge_plan_create_directed.restype = st
        lib.huge_plan_create_directed.argtypes = [vp, i32, i32, vp, vp, vp, ctypes.POINTER(ctypes.c_void_p)]
        lib.huge_count_paths.restype = st
        lib.huge_count_paths.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ExecOpts), vp]
        lib.huge_segment_rows.restype = st
        lib.huge_segment_rows.argtypes = [vp, vp, ctypes.POINTER(ExecOpts), vp]
        lib.huge_plan_bushy_nodes.restype = st
        lib.huge_plan_bushy_nodes.argtypes = [vp, ctypes.POINTER(BushyNode), i32, ctypes.POINTER(i32)]
        lib.huge_count_bushy.restype = st
        lib.huge_count_bushy.argtypes = [vp, vp, ctypes.POINTER(ExecOpts), ctypes.POINTER(Result), vp, i32]
        lib.huge_count_noalloc.restype = st
        lib.huge_count_noalloc.argtypes = [vp, vp, ctypes.POINTER(ExecOpts), ctypes.POINTER(Result)]
        lib.huge_noalloc_capacity.restype = st
        lib.huge_noalloc_capacity.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        lib.huge_workspace_size.restype = st
        lib.huge_workspace_size.argtypes = [vp, vp, ctypes.POINTER(ExecOpts), ctypes.POINTER(ctypes.c_uint64)]
        lib.huge_count.restype = st
        lib.huge_count.argtypes = [vp, vp, ctypes.POINTER(ExecOpts), ctypes.POINTER(Result)]
        lib.huge_enumerate.restype = st
        lib.huge_enumerate.argtypes = [vp, vp, ctypes.POINTER(ExecOpts), vp, i64, EMIT_FN, vp, ctypes.POINTER(Result)]
        lib.huge_count_batch.restype = st
        lib.huge_count_batch.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(ExecOpts), ctypes.POINTER(Result)]
        lib.huge_batch_workspace_size.restype = st
        lib.huge_batch_workspace_size.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(ExecOpts),
                                                  ctypes.POINTER(ctypes.c_uint64)]
        lib.huge_last_error.restype = ctypes.c_char_p
        lib.huge_last_error.argtypes = []
        f32, f64 = ctypes.c_float, ctypes.c_double
        lib.huge_model_create.restype = st
        lib.huge_model_create.argtypes = [ctypes.POINTER(vp)]
        lib.huge_model_free.restype = None
        lib.huge_model_free.argtypes = [vp]
        lib.huge_model_set.restype = st
        lib.huge_model_set.argtypes = [vp, vp, vp, vp, f32, f32]
        lib.huge_model_get.restype = st
        lib.huge_model_get.argtypes = [vp, vp, vp, vp, ctypes.POINTER(f32), ctypes.POINTER(f32)]
        lib.huge_model_forward.restype = st
        lib.huge_model_forward.argtypes = [vp, vp, i64, vp, vp]
        lib.huge_model_grad.restype = st
        lib.huge_model_grad.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(f64), vp]
        lib.huge_model_train.restype = st
        lib.huge_model_train.argtypes = [vp, vp, vp, i64, i32, i64, f32, ctypes.c_uint64, vp, vp]
        lib.huge_plan_features.restype = st
        lib.huge_plan_features.argtypes = [vp, vp, vp, i32, vp]
        lib.huge_autotune.restype = st
        lib.huge_autotune.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(ExecOpts), ctypes.POINTER(TuneTable)]
        lib.huge_graph_digest.restype = st
        lib.huge_graph_digest.argtypes = [vp, ctypes.c_char_p]
        lib.huge_device_name.restype = st
        lib.huge_device_name.argtypes = [ctypes.c_char_p, i32]
        lib.huge_plan_prefix.restype = st
        lib.huge_plan_prefix.argtypes = [vp, i32, ctypes.POINTER(vp)]
        lib.huge_plan_create_learned2.restype = st
        lib.huge_plan_create_learned2.argtypes = [vp, vp, i32, i32, vp, vp, u32, vp, ctypes.POINTER(vp)]
        lib.huge_plan_create_learned.restype = st
        lib.huge_plan_create_learned.argtypes = [vp, vp, i32, i32, vp, vp, vp, ctypes.POINTER(vp)]
        _lib = lib
        return lib


def _check(status):
    if status not in (HUGE_OK, HUGE_STOPPED):
        msg = _lib.huge_last_error()
        raise HugeError(status, msg.decode() if msg else "")
    return status


def _torch():
    import torch  # deferred: only needed for device memory and streams
    return torch


def _current_stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Graph:
    """A graph loaded on the current device (relabelled by degree rank)."""

    def __init__(self, handle, n, nnz):
        self._h = ctypes.c_void_p(handle)
        self.n = n
        self.nnz = nnz

    @property
    def handle(self):
        return self._h

    def info(self):
        gi = GraphInfo()
        _check(_lib.huge_graph_get_info(self._h, ctypes.byref(gi)))
        return {"n": gi.n, "nnz": gi.nnz, "max_degree": gi.max_degree,
                "degree_hist": [int(x) for x in gi.degree_hist],
                "degree_moments": [float(x) for x in gi.degree_moments], "load_ms": gi.load_ms,
                "device_bytes": int(gi.device_bytes), "hub_count": int(gi.hub_count),
                "hub_min_degree": int(gi.hub_min_degree)}

    def export(self):
        rp = np.empty(self.n + 1, dtype=np.int64)
        col = np.empty(max(self.nnz, 1), dtype=np.int32)
        inv = np.empty(self.n, dtype=np.int32)
        _check(_lib.huge_graph_export(self._h, rp.ctypes.data, col.ctypes.data, inv.ctypes.data))
        return rp, col[: self.nnz], inv

    def free(self):
        if self._h and self._h.value and _lib is not None:
            _lib.huge_graph_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plan:
    def __init__(self, handle, k, bushy=False):
        self._h = ctypes.c_void_p(handle)
        self.k = k
        self.bushy = bushy

    def bushy_nodes(self):
        """huge_plan_bushy_nodes: the join tree, children before parents, the root last."""
        n = ctypes.c_int32()
        out = (BushyNode * BUSHY_MAX_NODES)()
        _check(_lib.huge_plan_bushy_nodes(self._h, out, BUSHY_MAX_NODES, ctypes.byref(n)))
        return [{"edge_mask": int(x.edge_mask), "vertex_mask": int(x.vertex_mask), "kind": BUSHY_KINDS[x.kind],
                 "left": int(x.left), "right": int(x.right), "star_root": int(x.star_root),
                 "est_rows": float(x.est_rows), "cost": float(x.cost)} for x in out[: n.value]]

    @property
    def handle(self):
        return self._h

    def info(self):
        k = ctypes.c_int32()
        order = np.zeros(KMAX, dtype=np.int32)
        nsb = ctypes.c_int32()
        pairs = np.zeros(56, dtype=np.int32)
        est = ctypes.c_double()
        _check(_lib.huge_plan_info(self._h, ctypes.byref(k), order.ctypes.data, ctypes.byref(nsb),
                                   pairs.ctypes.data, ctypes.byref(est)))
        return {"k": k.value, "order": order[: k.value].tolist(),
                "sb_pairs": [tuple(pairs[2 * i:2 * i + 2].tolist()) for i in range(nsb.value)],
                "est_cost": est.value}

    def estimates(self):
        """huge_plan_estimates: estimated partial matches of each prefix size 1..k of the order."""
        est = np.zeros(KMAX, dtype=np.float64)
        _check(_lib.huge_plan_estimates(self._h, est.ctypes.data))
        return est[: self.k].tolist()

    def free(self):
        if self._h and self._h.value and _lib is not None:
            _lib.huge_plan_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def load(row_ptr, col, validate=True, stream=None, hub_bitmaps=True, labels=None) -> Graph:
    """huge_load_csr (or huge_load_csr_labelled with `labels`, one int per vertex).
    row_ptr/col: numpy arrays (host) or torch tensors on the GPU."""
    lib = load_library()
    flags = (0 if validate else NO_VALIDATE) | (0 if hub_bitmaps else NO_HUB_BITMAP)
    keep = []
    if hasattr(row_ptr, "is_cuda") and row_ptr.is_cuda:
        torch = _torch()
        rp = row_ptr.to(torch.int64).contiguous()
        cl = col.to(torch.int32).contiguous()
        keep += [rp, cl]
        n, nnz = rp.numel() - 1, cl.numel()
        flags |= DEVICE_PTRS
        prp, pcl = rp.data_ptr(), (cl.data_ptr() if nnz else None)
        s = stream if stream is not None else _current_stream()
    else:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        keep += [rp, cl]
        n, nnz = rp.shape[0] - 1, cl.shape[0]
        flags |= HOST_PTRS
        prp, pcl = rp.ctypes.data, (cl.ctypes.data if nnz else None)
        s = stream if stream is not None else _current_stream()
    h = ctypes.c_void_p()
    if labels is None:
        _check(lib.huge_load_csr(int(n), int(nnz), prp, pcl, flags, s, ctypes.byref(h)))
    else:
        if flags & DEVICE_PTRS:
            lb = labels.to(_torch().int32).contiguous()
            plb = lb.data_ptr()
        else:
            lb = np.ascontiguousarray(labels, dtype=np.int32)
            plb = lb.ctypes.data
        if lb.shape[0] != n:
            raise ValueError("labels must hold one entry per vertex")
        keep.append(lb)
        _check(lib.huge_load_csr_labelled(int(n), int(nnz), prp, pcl, plb, flags, s, ctypes.byref(h)))
    return Graph(h.value, int(n), int(nnz))


def plan(g: Graph, k, edges, order=None, learned=None, verify=False, induced=False, labels=None,
         all_maps=False) -> Plan:
    """huge_plan_create for query edges over vertices 0..k-1; with a Model as
    `learned`, huge_plan_create_learned2 (orders scored by the MLP on the GPU;
    verify=True measures its best orders on a small sample).  induced=True keeps
    only induced matches (HUGE_PLAN_INDUCED); labels (one int per query vertex,
    -1 any) plan a labelled query (huge_plan_create_labelled)."""
    lib = load_library()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    o = None if order is None else np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    h = ctypes.c_void_p()
    ind = (PLAN_INDUCED if induced else 0) | (PLAN_ALL_MAPS if all_maps else 0)  # all_maps: no symmetry breaking
    if labels is not None:
        if learned:
            raise ValueError("labelled queries are planned by the cost model")
        ql = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
        if ql.shape != (int(k),):
            raise ValueError("labels must hold one entry per query vertex")
        _check(lib.huge_plan_create_labelled(None if g is None else g.handle, int(k), int(e.shape[0]), e.ctypes.data,
                                             ql.ctypes.data, None if o is None else o.ctypes.data, ind,
                                             ctypes.byref(h)))
        return Plan(h.value, int(k))
    if isinstance(learned, Model):
        _check(lib.huge_plan_create_learned2(g.handle, learned.handle, int(k), int(e.shape[0]), e.ctypes.data,
                                             None if o is None else o.ctypes.data,
                                             (PLAN_VERIFY if verify else 0) | ind, _current_stream(), ctypes.byref(h)))
    else:
        _check(lib.huge_plan_create(None if g is None else g.handle, int(k), int(e.shape[0]), e.ctypes.data,
                                    None if o is None else o.ctypes.data,
                                    (PLAN_LEARNED if learned else PLAN_COST_MODEL) | ind, ctypes.byref(h)))
    return Plan(h.value, int(k))


def graph_info_struct(stats: dict) -> GraphInfo:
    """A huge_graph_info holding n, nnz and degree_moments from a dict (planning without a graph)."""
    gi = GraphInfo()
    gi.n, gi.nnz = int(stats["n"]), int(stats["nnz"])
    for i, m in enumerate(stats["degree_moments"]):
        gi.degree_moments[i] = float(m)
    return gi


def plan_bushy(g: Graph | None, k, edges, machines=1.0, stats: dict | None = None, labels=None,
               joins=None) -> Plan:
    """huge_plan_create_bushy: Algorithm 1's bushy plan; `machines` is its k (the
    pull cost k |E_G|); stats (n, nnz, degree_moments) plan without a graph.
    joins=[(left_mask, right_mask), ...] gives the tree instead
    (huge_plan_create_bushy_tree): masks over the query edges as listed."""
    lib = load_library()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    ql = None if labels is None else np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
    gi = None if stats is None else graph_info_struct(stats)
    h = ctypes.c_void_p()
    gh, gip = None if g is None else g.handle, None if gi is None else ctypes.byref(gi)
    qp = None if ql is None else ql.ctypes.data
    if joins is None:
        _check(lib.huge_plan_create_bushy(gh, gip, int(k), int(e.shape[0]), e.ctypes.data, qp, float(machines),
                                          ctypes.byref(h)))
    else:
        js = np.ascontiguousarray(np.asarray(joins, dtype=np.uint32).reshape(-1, 2))
        _check(lib.huge_plan_create_bushy_tree(gh, gip, int(k), int(e.shape[0]), e.ctypes.data, qp,
                                               js.ctypes.data if js.size else None, int(js.shape[0]),
                                               float(machines), ctypes.byref(h)))
    return Plan(h.value, int(k), bushy=True)


def load_directed(out_rp, out_col, hub_bitmaps=True, stream=None) -> Graph:
    """huge_load_csr_directed: a directed graph from its out-lists (host numpy arrays)."""
    lib = load_library()
    rp = np.ascontiguousarray(out_rp, dtype=np.int64)
    cl = np.ascontiguousarray(out_col, dtype=np.int32)
    n = int(rp.shape[0] - 1)
    h = ctypes.c_void_p()
    flags = HOST_PTRS | (0 if hub_bitmaps else NO_HUB_BITMAP)
    _check(lib.huge_load_csr_directed(n, int(cl.shape[0]), rp.ctypes.data, cl.ctypes.data if cl.size else None,
                                      flags, stream if stream is not None else _current_stream(), ctypes.byref(h)))
    gi = GraphInfo()
    _check(lib.huge_graph_get_info(h, ctypes.byref(gi)))
    return Graph(h.value, n, int(gi.nnz))


def plan_directed(g: Graph, k, arcs, order=None, labels=None) -> Plan:
    """huge_plan_create_directed: a directed query, arcs = [(a, b), ...] meaning a -> b."""
    lib = load_library()
    a = np.ascontiguousarray(np.asarray(arcs, dtype=np.int32).reshape(-1, 2))
    o = None if order is None else np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    ql = None if labels is None else np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
    h = ctypes.c_void_p()
    _check(lib.huge_plan_create_directed(None if g is None else g.handle, int(k), int(a.shape[0]), a.ctypes.data,
                                         None if ql is None else ql.ctypes.data, None if o is None else o.ctypes.data,
                                         ctypes.byref(h)))
    return Plan(h.value, int(k))


def count_paths(g: Graph, s: int, t: int, max_hops: int, **kw) -> list:
    """huge_count_paths: counts[L] = simple s-t paths of exactly L edges, L = 0..max_hops."""
    lib = load_library()
    opts = exec_opts(**kw)
    out = np.zeros(int(max_hops) + 1, dtype=np.uint64)
    _check(lib.huge_count_paths(g.handle, int(s), int(t), int(max_hops), ctypes.byref(opts), out.ctypes.data))
    return [int(x) for x in out]


def segment_rows(g: Graph, p: Plan, **kw) -> list:
    """huge_segment_rows: the level engine's rows per scheduling segment, per level."""
    lib = load_library()
    opts = exec_opts(**kw)
    rows = np.zeros(KMAX, dtype=np.int64)
    _check(lib.huge_segment_rows(g.handle, p.handle, ctypes.byref(opts), rows.ctypes.data))
    return rows.tolist()


def count_bushy(g: Graph, p: Plan, **kw):
    """huge_count_bushy: the result dict and the rows each tree node produced (-1
    for nodes inside a chain of pulled joins)."""
    lib = load_library()
    opts = exec_opts(**kw)
    r = Result()
    rows = np.full(BUSHY_MAX_NODES, -2, dtype=np.int64)
    _check(lib.huge_count_bushy(g.handle, p.handle, ctypes.byref(opts), ctypes.byref(r), rows.ctypes.data,
                                BUSHY_MAX_NODES))
    return r.to_dict(), rows.tolist()


def plan_features(g: Graph, p: Plan, size: int, order=None) -> np.ndarray:
    """huge_plan_features: the learned model's input for one order prefix."""
    lib = load_library()
    out = np.zeros(MLP_F, dtype=np.float32)
    o = None if order is None else np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    _check(lib.huge_plan_features(g.handle, p.handle, None if o is None else o.ctypes.data, int(size),
                                  out.ctypes.data))
    return out


class Model:
    """The learned cardinality model (huge_model_*): parameters live on the GPU."""

    def __init__(self):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.huge_model_create(ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set(self, params=None, xmean=None, xinv=None, tmean=0.0, tstd=1.0):
        arrs = []
        for a, n in ((params, MLP_PARAMS), (xmean, MLP_F), (xinv, MLP_F)):
            if a is None:
                arrs.append(None)
                continue
            a = np.ascontiguousarray(a, dtype=np.float32)
            if a.shape != (n,):
                raise ValueError("expected %d values, got shape %s" % (n, a.shape))
            arrs.append(a)
        _check(_lib.huge_model_set(self._h, *[None if a is None else a.ctypes.data for a in arrs],
                                   float(tmean), float(tstd)))
        return self

    def get(self):
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        xm = np.empty(MLP_F, dtype=np.float32)
        xi = np.empty(MLP_F, dtype=np.float32)
        tm, ts = ctypes.c_float(), ctypes.c_float()
        _check(_lib.huge_model_get(self._h, p.ctypes.data, xm.ctypes.data, xi.ctypes.data, ctypes.byref(tm),
                                   ctypes.byref(ts)))
        return {"params": p, "xmean": xm, "xinv": xi, "tmean": tm.value, "tstd": ts.value}

    @staticmethod
    def _dev(a):
        torch = _torch()
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()

    def forward(self, X) -> np.ndarray:
        torch = _torch()
        x = self._dev(np.asarray(X, dtype=np.float32).reshape(-1, MLP_F))
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(_lib.huge_model_forward(self._h, x.data_ptr(), int(x.shape[0]), y.data_ptr(), _current_stream()))
        torch.cuda.synchronize()
        return y.cpu().numpy()

    def grad(self, X, t):
        x = self._dev(np.asarray(X, dtype=np.float32).reshape(-1, MLP_F))
        tt = self._dev(np.asarray(t, dtype=np.float32).reshape(-1))
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        _check(_lib.huge_model_grad(self._h, x.data_ptr(), tt.data_ptr(), int(x.shape[0]), g.ctypes.data,
                                    ctypes.byref(loss), _current_stream()))
        return g, loss.value

    def train(self, X, t, epochs=100, batch=256, lr=1e-3, seed=0):
        x = self._dev(np.asarray(X, dtype=np.float32).reshape(-1, MLP_F))
        tt = self._dev(np.asarray(t, dtype=np.float32).reshape(-1))
        losses = np.empty(int(epochs), dtype=np.float32)
        _check(_lib.huge_model_train(self._h, x.data_ptr(), tt.data_ptr(), int(x.shape[0]), int(epochs), int(batch),
                                     float(lr), int(seed) & ((1 << 64) - 1), losses.ctypes.data, _current_stream()))
        return losses

    def save(self, path):
        d = self.get()
        np.savez(path, params=d["params"], xmean=d["xmean"], xinv=d["xinv"],
                 tnorm=np.array([d["tmean"], d["tstd"]], dtype=np.float32))

    @classmethod
    def load(cls, path):
        with np.load(path, allow_pickle=False) as z:
            m = cls()
            m.set(z["params"], z["xmean"], z["xinv"], float(z["tnorm"][0]), float(z["tnorm"][1]))
        return m

    def free(self):
        if self._h and self._h.value and _lib is not None:
            _lib.huge_model_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def exec_opts(cap=None, chunk_rows=0, strategy=-1, engine=ENGINE_AUTO, work_stealing=1, slice_count=1, slice_id=0,
              stream=None, workspace=None, profile=False, slice_vertex=0, hash=True, tune=None,
              work_limit=0, slice_mode=SLICE_MIX, slice2=None) -> ExecOpts:
    """huge_exec_opts from keywords; slice2=(query vertex, count, id) is the second vertex slice,
    slice2=(a, b, count, id) a second slice on the pair of adjacent query vertices (a, b)."""
    lib = load_library()
    o = ExecOpts()
    lib.huge_exec_opts_default(ctypes.byref(o))
    if cap is not None:
        o.frontier_cap_bytes = (1 << 64) - 1 if cap == float("inf") else int(cap)
    o.chunk_rows = int(chunk_rows)
    o.strategy = int(strategy)
    o.engine = int(engine)
    o.work_stealing = int(work_stealing)
    o.slice_count = int(slice_count)
    o.slice_id = int(slice_id)
    o.profile = 1 if profile else 0
    o.slice_vertex = int(slice_vertex)
    o.exec_flags = 0 if hash else EXEC_NO_HASH
    o.work_limit = int(work_limit)
    o.slice_mode = int(slice_mode)
    if slice2 is not None:
        if len(slice2) == 4:
            o.slice2_vertex, o.slice2_vertex2 = int(slice2[0]), int(slice2[1])
            o.exec_flags |= EXEC_SLICE2_PAIR
        else:
            o.slice2_vertex = int(slice2[0])
        o.slice2_count, o.slice2_id = int(slice2[-2]), int(slice2[-1])
    if tune is not None:
        o.tune = ctypes.cast(ctypes.byref(tune), ctypes.c_void_p)
    o.stream = (stream if stream is not None else _current_stream()).value \
        if not isinstance(stream, int) else stream
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


class Workspace:
    """A grow-only device buffer (torch-owned) reused across exec calls."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        return self.buf


_default_ws = Workspace()


def workspace_size(g: Graph, p: Plan, opts: ExecOpts) -> int:
    b = ctypes.c_uint64()
    _check(_lib.huge_workspace_size(g.handle, p.handle, ctypes.byref(opts), ctypes.byref(b)))
    return int(b.value)


def count(g: Graph, p: Plan, workspace: Workspace | None = _default_ws, **kw) -> dict:
    """huge_count: count matches; returns count, hash_sum, hash_xor, level_counts, query_ms, ..."""
    lib = load_library()
    opts = exec_opts(**kw)
    if workspace is not None and not getattr(p, "bushy", False):  # bushy plans allocate their own tables
        ws = workspace.get(workspace_size(g, p, opts))
        opts.workspace = ws.data_ptr()
        opts.workspace_bytes = ws.numel()
    r = Result()
    status = _check(lib.huge_count(g.handle, p.handle, ctypes.byref(opts), ctypes.byref(r)))
    d = r.to_dict()
    d["stopped"] = status == HUGE_STOPPED
    return d


def motif_count(g: Graph, k: int, **kw) -> list:
    """huge_motif_count: every connected k-vertex pattern with its non-induced count
    (and set-hashes) and induced count, as dicts."""
    lib = load_library()
    opts = exec_opts(**kw)
    out = (Motif * MOTIF_MAX)()
    n = ctypes.c_int32()
    _check(lib.huge_motif_count(g.handle, int(k), ctypes.byref(opts), out, ctypes.byref(n)))
    return [{"k": m.k, "edges": [(m.edges[2 * i], m.edges[2 * i + 1]) for i in range(m.n_edges)],
             "noninduced": int(m.noninduced), "induced": int(m.induced), "hash_sum": int(m.hash_sum),
             "hash_xor": int(m.hash_xor)} for m in out[: n.value]]


def count_noalloc(g: Graph, p: Plan, **kw) -> dict:
    """huge_count_noalloc: huge_count in the library's own fixed device array (no allocation)."""
    lib = load_library()
    opts = exec_opts(**kw)
    r = Result()
    status = _check(lib.huge_count_noalloc(g.handle, p.handle, ctypes.byref(opts), ctypes.byref(r)))
    d = r.to_dict()
    d["stopped"] = status == HUGE_STOPPED
    return d


def noalloc_capacity() -> int:
    lib = load_library()
    b = ctypes.c_uint64()
    _check(lib.huge_noalloc_capacity(ctypes.byref(b)))
    return int(b.value)


def plan_prefix(p: Plan, size: int) -> Plan:
    """huge_plan_prefix: the plan of the first `size` order vertices of p."""
    lib = load_library()
    h = ctypes.c_void_p()
    _check(lib.huge_plan_prefix(p.handle, int(size), ctypes.byref(h)))
    return Plan(h.value, int(size))


def graph_digest(g: Graph) -> str:
    lib = load_library()
    buf = ctypes.create_string_buffer(65)
    _check(lib.huge_graph_digest(g.handle, buf))
    return buf.value.decode()


def device_name() -> str:
    """huge_device_name: architecture and compute units of the current device."""
    lib = load_library()
    buf = ctypes.create_string_buffer(128)
    _check(lib.huge_device_name(buf, 128))
    return buf.value.decode()


def autotune(g: Graph, plans, cache=None, **kw) -> TuneTable:
    """huge_autotune on a sample chosen by the slice options in kw; with `cache` (a JSON file), the
    table is stored under (graph digest, GPU name) and reused when present."""
    import json

    lib = load_library()
    key = None
    if cache is not None:
        key = "%s|%s" % (graph_digest(g), device_name())
        if os.path.exists(cache):
            with open(cache) as f:
                d = json.load(f)
            if key in d:
                return TuneTable.from_dict(d[key])
    opts = exec_opts(**kw)
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    t = TuneTable()
    _check(lib.huge_autotune(g.handle, arr, len(plans), ctypes.byref(opts), ctypes.byref(t)))
    if cache is not None:
        d = {}
        if os.path.exists(cache):
            with open(cache) as f:
                d = json.load(f)
        d[key] = t.to_dict()
        with open(cache, "w") as f:
            json.dump(d, f, indent=1)
    return t


def count_batch(g: Graph, plans, workspace: Workspace | None = None, **kw):
    """huge_count_batch; with engine=ENGINE_GRAPH a Workspace holds the batch's device memory."""
    lib = load_library()
    opts = exec_opts(**kw)
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    if workspace is not None and opts.engine == ENGINE_GRAPH:
        b = ctypes.c_uint64()
        _check(lib.huge_batch_workspace_size(g.handle, arr, len(plans), ctypes.byref(opts), ctypes.byref(b)))
        ws = workspace.get(int(b.value))
        opts.workspace = ws.data_ptr()
        opts.workspace_bytes = ws.numel()
    res = (Result * len(plans))()
    _check(lib.huge_count_batch(g.handle, arr, len(plans), ctypes.byref(opts), res))
    return [r.to_dict() for r in res]


def enumerate_matches(g: Graph, p: Plan, buf_rows=1 << 16, callback=None, **kw):
    """huge_enumerate.  Returns the result dict; with callback None it also holds
    every match under "rows", an (N, k) int32 array (query-vertex order, original
    IDs).  Otherwise callback(rows) is called per buffer and a true return stops."""
    lib = load_library()
    opts = exec_opts(**kw)
    buf = np.empty((int(buf_rows), p.k), dtype=np.int32)
    chunks = []

    def _cb(user, rows, nrows, k):
        a = np.ctypeslib.as_array(rows, shape=(int(nrows) * int(k),)).reshape(int(nrows), int(k)).copy()
        if callback is None:
            chunks.append(a)
            return 0
        return 1 if callback(a) else 0

    fn = EMIT_FN(_cb)
    r = Result()
    st = _check(lib.huge_enumerate(g.handle, p.handle, ctypes.byref(opts), buf.ctypes.data, int(buf_rows), fn, None,
                                   ctypes.byref(r)))
    d = r.to_dict()
    d["stopped"] = st == HUGE_STOPPED
    if callback is None:
        d["rows"] = np.concatenate(chunks) if chunks else np.zeros((0, p.k), dtype=np.int32)
    return d
