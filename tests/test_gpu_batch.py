"""Concurrent batches on the level engine (huge_count_batch with several
streams): every query's result equals its single run and the oracle."""
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def graph(H):
    g = gg.chung_lu(2500, 9, 2.4, seed=41)
    return g, H.load(g.row_ptr, g.col)


def test_concurrent_batch_matches_oracle(H, graph):
    g, G = graph
    pats = P.random_patterns(24, seed=8, kmin=3, kmax=6)
    plans = [H.plan(G, p["k"], p["edges"]) for p in pats]
    outs = H.count_batch(G, plans)
    assert len(outs) == len(plans)
    for p, pl, r in zip(pats, plans, outs):
        ref = oracle_run(g, p["k"], p["edges"], order=pl.info()["order"])
        assert cmp_key(r, p["k"]) == cmp_key(ref, p["k"]), p
        assert r["level_counts"][:p["k"]] == ref["level_counts"][:p["k"]], p


def test_concurrent_batch_with_slices_and_table(H, graph):
    g, G = graph
    names = ["triangle", "4-cycle", "diamond", "house", "5-clique", "6-cycle", "tailed-triangle", "4-path"]
    plans = [H.plan(G, *P.NAMED[n]) for n in names]
    t = H.TuneTable()
    for j in range(H.KMAX + 1):
        for c in range(H.TUNE_BUCKETS):
            t.strategy[j][c] = (j + c) % H.STRAT_COUNT
    for s in range(2):
        outs = H.count_batch(G, plans, slice_count=2, slice_id=s, slice_vertex=-1, tune=t, cap=0)
        for n, pl, r in zip(names, plans, outs):
            single = H.count(G, pl, slice_count=2, slice_id=s, slice_vertex=-1)
            k = P.NAMED[n][0]
            assert cmp_key(r, k) == cmp_key(single, k), (n, s)


def test_concurrent_batch_reports_errors(H, graph):
    _, G = graph
    plans = [H.plan(G, *P.NAMED[n]) for n in ["triangle", "diamond", "house"]]
    with pytest.raises(RuntimeError, match="slice_id"):
        H.count_batch(G, plans, slice_count=2, slice_id=5)
