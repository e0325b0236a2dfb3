"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (per-bucket dispatch with several kernels, the workloads'
frontier caps and slicing), on sampled outputs the oracle recomputes one by
one: small root slices (on each plan's first matched vertex) of the R-MAT 22
and Chung-Lu 3.07M graphs, and small edge slices of the R-MAT 24 and 26
graphs."""
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu, oracle_run

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def H():
    return need_gpu()


def _table(H):
    """A mixed dispatch like the tuned ones: binary search, 4-, 16- and 64-wide
    lane merge, and both block-cached lane merges."""
    t = H.TuneTable()
    rows = {1: [3, 3, 3, 3, 3], 2: [0, 4, 6, 6, 6], 3: [2, 5, 4, 6, 6], 4: [0, 2, 5, 6, 4]}
    for j in range(H.KMAX + 1):
        for c in range(H.TUNE_BUCKETS):
            t.strategy[j][c] = rows.get(j, [2] * 5)[c]
    return t


def _check(H, G, g, names, S, ids, edge, cap):
    t = _table(H)
    for name in names:
        k, e = P.NAMED[name]
        p = H.plan(G, k, e)
        order = p.info()["order"]
        for s in ids:
            r = H.count(G, p, tune=t, cap=cap, slice_count=S, slice_id=s, slice_vertex=-2 if edge else -1)
            okw = {"slice_pair": (order[0], order[1])} if edge else {"slice_vertex": order[0]}
            ref = oracle_run(g, k, e, order=order, slice_count=S, slice_id=s, **okw)
            assert cmp_key(r, k) == cmp_key(ref, k), (name, s)
            assert r["level_counts"][1:k] == ref["level_counts"][1:k], (name, s)


def test_rmat22_root_slices(H):
    g = gg.rmat(22, 16, seed=2)
    G = H.load(g.row_ptr, g.col)
    _check(H, G, g, ["4-clique", "diamond", "4-cycle"], 1 << 18, [0, 77], edge=False, cap=4 << 30)


def test_chung_lu_3m_root_slices(H):
    g = gg.chung_lu(3072441, 76, 2.2, seed=3)
    G = H.load(g.row_ptr, g.col)
    _check(H, G, g, ["5-clique", "house"], 1 << 19, [0, 5], edge=False, cap=32 << 30)


def test_rmat24_edge_slices(H):
    g = gg.rmat(24, 16, seed=4)
    G = H.load(g.row_ptr, g.col)
    _check(H, G, g, ["4-cycle", "diamond", "tailed-triangle"], 1 << 24, [0, 3], edge=True, cap=8 << 30)


def test_rmat26_edge_slices(H):
    g = gg.rmat(26, 16, seed=5)
    G = H.load(g.row_ptr, g.col)
    _check(H, G, g, ["4-clique", "4-cycle"], 1 << 26, [0], edge=True, cap=16 << 30)
