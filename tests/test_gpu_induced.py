"""Induced matching (HUGE_PLAN_INDUCED): only matches whose image is an induced
subgraph (every non-edge of q maps to a non-edge of G), against the oracle's
induced mode, on every engine and strategy, and against closed forms."""
import math

import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu

NAMES = ["wedge", "4-path", "3-star", "4-cycle", "tailed-triangle", "diamond", "5-cycle", "house", "6-cycle"]


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def graph(H):
    g = gg.chung_lu(2500, 10, 2.3, seed=81)
    return g, H.load(g.row_ptr, g.col)


@pytest.mark.parametrize("name", NAMES)
def test_induced_matches_oracle(H, graph, name):
    g, G = graph
    k, e = P.NAMED[name]
    p = H.plan(G, k, e, induced=True)
    order = p.info()["order"]
    ref = oracle_run(g, k, e, order=order, induced=True)
    for strategy in range(H.STRAT_COUNT):
        r = H.count(G, p, strategy=strategy)
        assert cmp_key(r, k) == cmp_key(ref, k), (name, strategy)
        assert r["level_counts"][:k] == ref["level_counts"][:k], (name, strategy)
    r = H.count(G, p, engine=H.ENGINE_GRAPH)
    assert cmp_key(r, k) == cmp_key(ref, k), name
    plain = H.count(G, H.plan(G, k, e))
    assert r["count"] <= plain["count"]


def test_induced_batched_slices_and_hubs(H):
    g = gg.rmat(11, 16, seed=82)
    G = H.load(g.row_ptr, g.col)
    pats = P.random_patterns(12, seed=83, kmin=3, kmax=5)
    plans = [H.plan(G, p["k"], p["edges"], induced=True) for p in pats]
    outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, slice_count=4, slice_id=1, slice_vertex=-1,
                         slice_mode=H.SLICE_STRIDE)
    for p, pl, r in zip(pats, plans, outs):
        o = pl.info()["order"]
        ref = oracle_run(g, p["k"], p["edges"], order=o, induced=True, slice_count=4, slice_id=1,
                         slice_vertex=o[0], slice_mode=1)
        assert cmp_key(r, p["k"]) == cmp_key(ref, p["k"]), p


def test_induced_closed_forms(H):
    K = gg.complete(8)
    G = H.load(K.row_ptr, K.col)
    assert H.count(G, H.plan(G, *P.NAMED["4-clique"], induced=True))["count"] == math.comb(8, 4)
    for name in ["4-cycle", "diamond", "4-path", "house"]:
        assert H.count(G, H.plan(G, *P.NAMED[name], induced=True))["count"] == 0, name
    C = gg.cycle(9)
    Gc = H.load(C.row_ptr, C.col)
    assert H.count(Gc, H.plan(Gc, *P.NAMED["4-path"], induced=True))["count"] == 9
    assert H.count(Gc, H.plan(Gc, *P.NAMED["3-star"], induced=True))["count"] == 0
    with pytest.raises(H.HugeError):
        H.count(G, H.plan(G, *P.NAMED["4-cycle"], induced=True), engine=H.ENGINE_PERSISTENT)
