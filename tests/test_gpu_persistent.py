"""GPU parity of the persistent engine (per-workgroup Algorithm 5 with work
stealing) and of batched multi-query launches, against the oracle."""
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import assert_parity, cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu

PERSIST = 2


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def small(H):
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    return g, H.load(g.row_ptr, g.col)


@pytest.mark.parametrize("steal", [1, 0])
@pytest.mark.parametrize("name", ["triangle", "4-cycle", "diamond", "4-clique", "house", "5-clique", "tailed-triangle",
                                  "5-cycle", "6-cycle"])
def test_persistent_named(H, small, name, steal):
    g, G = small
    k, e = P.NAMED[name]
    r, ref = assert_parity(H, G, g, k, e, engine=PERSIST, work_stealing=steal)
    assert r["count"] > 0


def test_persistent_small_frontier_steals(H, small):
    """A small frontier budget keeps per-workgroup levels short, so rows move between workgroups."""
    g, G = small
    for name in ["house", "5-clique", "4-cycle"]:
        k, e = P.NAMED[name]
        r, _ = assert_parity(H, G, g, k, e, engine=PERSIST, cap=0)
    big = gg.rmat(12, 16, seed=4)
    Gb = H.load(big.row_ptr, big.col)
    k, e = P.NAMED["4-cycle"]
    a = H.count(Gb, H.plan(Gb, k, e), engine=PERSIST, cap=0)
    b = H.count(Gb, H.plan(Gb, k, e))
    assert cmp_key(a, k) == cmp_key(b, k)
    assert a["level_counts"][:k] == b["level_counts"][:k]


def test_persistent_slices(H, small):
    g, G = small
    k, e = P.NAMED["house"]
    for s in range(3):
        assert_parity(H, G, g, k, e, engine=PERSIST, slice_count=3, slice_id=s, slice_vertex=1)


def test_batched_patterns_match_single_runs(H):
    g = gg.chung_lu(2000, 8, 2.5, seed=33)
    G = H.load(g.row_ptr, g.col)
    pats = P.random_patterns(16, seed=3, kmin=3, kmax=5)
    plans = [H.plan(G, p["k"], p["edges"]) for p in pats]
    outs = H.count_batch(G, plans)
    for p, pl, r in zip(pats, plans, outs):
        ref = oracle_run(g, p["k"], p["edges"], order=pl.info()["order"])
        assert cmp_key(r, p["k"]) == cmp_key(ref, p["k"]), p
        assert r["level_counts"][:p["k"]] == ref["level_counts"][:p["k"]], p
