"""GPU parity at the edges of the input space: the largest queries (7 and 8
vertices), empty and edgeless graphs, isolated vertices, graphs that are a
single edge, and query shapes with closed-form counts on named graphs."""
import math

import numpy as np
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import assert_parity, cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    return need_gpu()


def _cycle_q(k):
    return k, [(i, (i + 1) % k) for i in range(k)]


def _path_q(k):
    return k, [(i, i + 1) for i in range(k - 1)]


def _clique_q(k):
    return k, [(a, b) for a in range(k) for b in range(a + 1, k)]


@pytest.mark.parametrize("q", [_cycle_q(7), _cycle_q(8), _path_q(7), _path_q(8), _clique_q(7), _clique_q(8)],
                         ids=["7-cycle", "8-cycle", "7-path", "8-path", "7-clique", "8-clique"])
def test_largest_queries(H, q):
    k, e = q
    g = gg.gnp(14, 0.55, seed=k + len(e))
    G = H.load(g.row_ptr, g.col)
    assert_parity(H, G, g, k, e)
    assert_parity(H, G, g, k, e, cap=0)


def test_largest_queries_closed_forms(H):
    n = 11
    g = gg.complete(n)
    G = H.load(g.row_ptr, g.col)
    for k in (7, 8):
        r = H.count(G, H.plan(G, *_clique_q(k)))
        assert r["count"] == math.comb(n, k)
        r = H.count(G, H.plan(G, *_path_q(k)))
        assert r["count"] == math.perm(n, k) // 2
        r = H.count(G, H.plan(G, *_cycle_q(k)))
        assert r["count"] == math.perm(n, k) // (2 * k)
    c = gg.cycle(8)
    Gc = H.load(c.row_ptr, c.col)
    assert H.count(Gc, H.plan(Gc, *_cycle_q(8)))["count"] == 1
    assert H.count(Gc, H.plan(Gc, *_path_q(8)))["count"] == 8


def test_edgeless_and_isolated(H):
    # no edges at all
    rp = np.zeros(6, dtype=np.int64)
    G = H.load(rp, np.zeros(0, dtype=np.int32))
    for name in ["edge", "triangle", "4-cycle", "house"]:
        k, e = P.NAMED[name]
        r = H.count(G, H.plan(G, k, e))
        assert r["count"] == 0 and r["hash_sum"] == 0 and r["hash_xor"] == 0
    # a triangle plus isolated vertices, and a lone edge
    g = gg.from_edges(9, [(0, 1), (1, 2), (0, 2), (5, 7)], permute=True, seed=3)
    G = H.load(g.row_ptr, g.col)
    for name in ["edge", "triangle", "wedge", "4-cycle", "4-path"]:
        k, e = P.NAMED[name]
        assert_parity(H, G, g, k, e)
    assert H.count(G, H.plan(G, *P.NAMED["edge"]))["count"] == 4
    assert H.count(G, H.plan(G, *P.NAMED["triangle"]))["count"] == 1


def test_single_edge_graph(H):
    g = gg.from_edges(2, [(0, 1)])
    G = H.load(g.row_ptr, g.col)
    assert_parity(H, G, g, *P.NAMED["edge"])
    assert H.count(G, H.plan(G, *P.NAMED["triangle"]))["count"] == 0
    rows = H.enumerate_matches(G, H.plan(G, *P.NAMED["edge"]), buf_rows=4)["rows"]
    assert sorted(map(tuple, rows.tolist())) in ([(0, 1)], [(1, 0)])


def test_slices_with_more_slices_than_vertices(H):
    g = gg.chung_lu(300, 6, 2.5, seed=9)
    G = H.load(g.row_ptr, g.col)
    k, e = P.NAMED["4-cycle"]
    full = H.count(G, H.plan(G, k, e))
    tot = 0
    for s in range(1024):
        tot += H.count(G, H.plan(G, k, e), slice_count=1024, slice_id=s)["count"]
    assert tot == full["count"]
