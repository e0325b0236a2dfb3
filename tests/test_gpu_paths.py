"""Hop-constrained s-t path counts (Section 6's path queries) and all-map plans
on the GPU, against the oracle's pinned all-maps path queries (pinned in
tests/test_oracle_pins.py against a depth-first search and K_n's closed form)."""
import math

import pytest

import graphgen as gg
import oracle
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu
from tests.test_oracle_pins import pinned_path_counts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    return need_gpu()


def test_paths_on_complete_graphs(H):
    K = gg.complete(9)
    G = H.load(K.row_ptr, K.col)
    for eng in (H.ENGINE_LEVELS, H.ENGINE_GRAPH):
        assert H.count_paths(G, 1, 6, 7, engine=eng) == [0] + [math.factorial(7) // math.factorial(8 - L)
                                                              for L in range(1, 8)]


@pytest.mark.parametrize("graph", ["cl", "rmat"])
def test_paths_match_oracle(H, graph):
    g = gg.chung_lu(2000, 8, 2.4, seed=81) if graph == "cl" else gg.rmat(10, 6, seed=82)
    G = H.load(g.row_ptr, g.col)
    rk = oracle.ranks(g.row_ptr)
    deg = [int(g.row_ptr[u + 1] - g.row_ptr[u]) for u in range(g.n)]
    hubs = sorted(range(g.n), key=lambda u: -deg[u])
    pairs = [(hubs[0], hubs[1]), (hubs[5], hubs[40]), (hubs[100], hubs[3])]
    for s, t in pairs:
        want = pinned_path_counts(g, s, t, 5, ranks=rk)
        for eng in (H.ENGINE_LEVELS, H.ENGINE_GRAPH):
            assert H.count_paths(G, s, t, 5, engine=eng) == want, (graph, s, t, eng)
    # the paths do not depend on the direction they are read in
    s, t = pairs[1]
    assert H.count_paths(G, s, t, 4) == H.count_paths(G, t, s, 4)


def test_all_maps_plans(H):
    """HUGE_PLAN_ALL_MAPS drops the symmetry-breaking constraints: every
    injective map is counted, |Aut(q)| per subgraph."""
    g = gg.chung_lu(1500, 10, 2.4, seed=83)
    G = H.load(g.row_ptr, g.col)
    for name in ["triangle", "4-cycle", "diamond", "house"]:
        k, e = P.NAMED[name]
        r = H.count(G, H.plan(G, k, e, all_maps=True))
        assert r["count"] == H.count(G, H.plan(G, k, e))["count"] * len(oracle.automorphisms(k, e)), name
        ref = oracle.enumerate_query(g.row_ptr, g.col, k, e, mode=oracle.MODE_ALL)
        assert cmp_key(r, k) == cmp_key(ref, k), name


def test_path_errors(H):
    g = gg.chung_lu(300, 6, 2.5, seed=84)
    G = H.load(g.row_ptr, g.col)
    for bad in [dict(s=1, t=1, max_hops=3), dict(s=0, t=1, max_hops=0), dict(s=0, t=1, max_hops=8),
                dict(s=-1, t=1, max_hops=3), dict(s=0, t=1, max_hops=3, slice_count=4)]:
        kw = dict(bad)
        s, t, h = kw.pop("s"), kw.pop("t"), kw.pop("max_hops")
        with pytest.raises(H.HugeError) as ei:
            H.count_paths(G, s, t, h, **kw)
        assert ei.value.name == "HUGE_EINVAL", bad
