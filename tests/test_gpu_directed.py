"""Directed graphs and queries (Section 2: the techniques carry over to directed
graphs) against the oracle's directed enumerator: the engines search the
undirected skeleton and keep every query edge's direction by lookups in the
out-lists.  Covers one-way and reciprocated query edges, every order of a
query, both engines, batches, slices, undirected queries on a directed
graph (they match its skeleton) and the errors."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_common import cmp_key, need_gpu

pytestmark = pytest.mark.gpu

QUERIES = {
    "cycle3": (3, [(0, 1), (1, 2), (2, 0)]),
    "transitive3": (3, [(0, 1), (1, 2), (0, 2)]),
    "path2": (3, [(0, 1), (1, 2)]),
    "recip-tail": (3, [(0, 1), (1, 0), (1, 2)]),
    "in-star": (4, [(1, 0), (2, 0), (3, 0)]),
    "bifan": (4, [(0, 2), (0, 3), (1, 2), (1, 3)]),
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "ffl-diamond": (4, [(0, 1), (0, 2), (1, 3), (2, 3), (1, 2)]),
    "recip-triangle": (3, [(0, 1), (1, 0), (1, 2), (2, 1), (0, 2)]),
    "cycle5-chord": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 2)]),
    "edge": (2, [(0, 1)]),
    "mutual": (2, [(0, 1), (1, 0)]),
}


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def graphs(H):
    out = {}
    for name, base, pb in [("cl", gg.chung_lu(1500, 10, 2.4, seed=71), 0.2), ("rmat", gg.rmat(10, 8, seed=72), 0.35)]:
        d = gg.orient(base, pb, seed=73)
        out[name] = (d, H.load_directed(d.out_rp, d.out_col))
    return out


def ref(d, k, e, **kw):
    return oracle.enumerate_directed(d.row_ptr, d.col, d.out_rp, d.out_col, k, e, **kw)


@pytest.mark.parametrize("name", sorted(QUERIES))
def test_directed_queries_match_oracle(H, graphs, name):
    k, e = QUERIES[name]
    for gname, (d, G) in graphs.items():
        p = H.plan_directed(G, k, e)
        want = ref(d, k, e)
        for eng in (H.ENGINE_LEVELS, H.ENGINE_GRAPH):
            r = H.count(G, p, engine=eng)
            assert cmp_key(r, k) == cmp_key(want, k), (name, gname, eng, r["count"], want["count"])
        order = p.info()["order"]
        lv = ref(d, k, e, order=order)["level_counts"]
        assert H.count(G, p)["level_counts"][1:k] == lv[1:k], (name, gname)


@pytest.mark.parametrize("name", ["transitive3", "bifan", "ffl-diamond", "cycle5-chord"])
def test_every_order_and_small_queues(H, graphs, name):
    d, G = graphs["rmat"]
    k, e = QUERIES[name]
    want = cmp_key(ref(d, k, e), k)
    adj = {(a, b) for a, b in e} | {(b, a) for a, b in e}
    for o in itertools.permutations(range(k)):
        if not all(any((o[i], o[j]) in adj for j in range(i)) for i in range(1, k)):
            continue
        p = H.plan_directed(G, k, e, order=list(o))
        assert cmp_key(H.count(G, p), k) == want, (name, o)
    p = H.plan_directed(G, k, e)
    assert cmp_key(H.count(G, p, cap=0, chunk_rows=64), k) == want


def test_directed_batches_slices_and_labels(H, graphs):
    d, G = graphs["cl"]
    names = ["cycle3", "transitive3", "bifan", "cycle4", "recip-tail", "ffl-diamond"]
    plans = [H.plan_directed(G, *QUERIES[n]) for n in names]
    for eng in (H.ENGINE_GRAPH, H.ENGINE_AUTO):
        outs = H.count_batch(G, plans, engine=eng)
        for n, r in zip(names, outs):
            k, e = QUERIES[n]
            assert cmp_key(r, k) == cmp_key(ref(d, k, e), k), (n, eng)
    k, e = QUERIES["bifan"]
    p = H.plan_directed(G, k, e)
    for mode in (H.SLICE_MIX, H.SLICE_STRIDE):
        tot = [0, 0, 0]
        for s in range(4):
            r = H.count(G, p, slice_count=4, slice_id=s, slice_vertex=2, slice_mode=mode)
            want = ref(d, k, e, slice_count=4, slice_id=s, slice_vertex=2, slice_mode=int(mode))
            assert cmp_key(r, k) == cmp_key(want, k), (mode, s)
            tot = [tot[0] + r["count"], (tot[1] + r["hash_sum"]) % (1 << 64), tot[2] ^ r["hash_xor"]]
        assert tuple(tot) == cmp_key(ref(d, k, e), k)
    # directed graphs carry no labels: a labelled directed query is refused
    with pytest.raises(H.HugeError) as ei:
        H.count(G, H.plan_directed(G, 3, QUERIES["cycle3"][1], labels=[0, 1, 2]))
    assert ei.value.name == "HUGE_EINVAL"


def test_undirected_queries_match_the_skeleton(H, graphs):
    from graphgen import patterns as P

    d, G = graphs["rmat"]
    for name in ["triangle", "4-cycle", "diamond"]:
        k, e = P.NAMED[name]
        r = H.count(G, H.plan(G, k, e))
        assert cmp_key(r, k) == cmp_key(oracle.enumerate_query(d.row_ptr, d.col, k, e), k), name


def test_directed_errors(H, graphs):
    d, G = graphs["cl"]
    u = gg.chung_lu(300, 6, 2.5, seed=74)
    Gu = H.load(u.row_ptr, u.col)
    p = H.plan_directed(G, *QUERIES["cycle3"])
    with pytest.raises(H.HugeError) as ei:
        H.count(Gu, p)  # a directed query on an undirected graph
    assert ei.value.name == "HUGE_EINVAL"
    with pytest.raises(H.HugeError) as ei:
        H.count(G, p, engine=H.ENGINE_PERSISTENT)
    assert ei.value.name == "HUGE_EINVAL"
    for bad in ([(0, 1), (0, 1)], [(0, 0)], [(0, 1), (2, 3)]):
        with pytest.raises(H.HugeError) as ei:
            H.plan_directed(G, 4 if bad == [(0, 1), (2, 3)] else 2, bad)
        assert ei.value.name == "HUGE_EQUERY", bad
    bad_graph = [(np.array([0, 1, 1]), np.array([0])),       # self-loop
                 (np.array([0, 2, 2, 2]), np.array([2, 1])),  # unsorted
                 (np.array([0, 1, 1]), np.array([5]))]         # out of range
    for rp, col in bad_graph:
        with pytest.raises(H.HugeError) as ei:
            H.load_directed(rp, col)
        assert ei.value.name == "HUGE_EGRAPH", (rp, col)
