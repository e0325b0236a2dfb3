"""Batched rounds (huge_count_batch on the graph engine): every query keeps its
own device scheduler state and the round's launches serve all queries; each
result equals the oracle and the query's own huge_count, bit for bit."""
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
    g = gg.chung_lu(700, 6, 2.4, seed=41)
    return g, H.load(g.row_ptr, g.col)


@pytest.fixture(scope="module")
def hubs(H):
    g = gg.rmat(9, 16, seed=43)
    return g, H.load(g.row_ptr, g.col)


def _check_all(H, g, pats, plans, outs, **okw):
    assert len(outs) == len(plans)
    for p, pl, r in zip(pats, plans, outs):
        ref = oracle_run(g, p["k"], p["edges"], order=pl.info()["order"], **okw)
        assert cmp_key(r, p["k"]) == cmp_key(ref, p["k"]), p
        assert r["level_counts"][:p["k"]] == ref["level_counts"][:p["k"]], p


def test_batched_rounds_match_oracle(H, graph):
    g, G = graph
    pats = P.random_patterns(36, seed=8, kmin=2, kmax=6)
    pats.append({"k": 7, "edges": [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 6), (6, 0), (0, 3)]})
    plans = [H.plan(G, p["k"], p["edges"]) for p in pats]
    print("batched rounds: %d queries" % len(plans), flush=True)
    outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH)
    _check_all(H, g, pats, plans, outs)


@pytest.mark.parametrize("cap,chunk,strategy", [(0, 0, -1), (1 << 20, 300, 2), (1 << 24, 4096, 3),
                                                (0, 500, 4), (1 << 22, 0, 5), (0, 64, 6), (0, 300, 0),
                                                (1 << 24, 0, 0), (1 << 20, 64, 1)])
def test_batched_rounds_small_queues_and_strategies(H, hubs, cap, chunk, strategy):
    """Hub-heavy R-MAT, tiny frontier caps (many yields and backtracks per query),
    small segments and every strategy (lane merges; 0 and 1 run binary-search
    tiles): equal to single runs."""
    g, G = hubs
    names = ["triangle", "4-cycle", "diamond", "house", "5-cycle", "tailed-triangle", "4-clique"]
    if cap >= (1 << 24):
        names.append("6-cycle")  # ~2e9 matches: with 4096-row queues this is ~1e5 rounds
    plans = [H.plan(G, *P.NAMED[n]) for n in names]
    print("batched rounds hubs cap=%d chunk=%d strategy=%d" % (cap, chunk, strategy), flush=True)
    outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, cap=cap, chunk_rows=chunk, strategy=strategy)
    for n, pl, r in zip(names, plans, outs):
        k = P.NAMED[n][0]
        single = H.count(G, pl)
        assert cmp_key(r, k) == cmp_key(single, k), n
        assert r["level_counts"][:k] == single["level_counts"][:k], n
        assert r["level_work"][:k] == single["level_work"][:k], n
        if cap:
            assert r["peak_frontier_bytes"] <= cap // len(names) + (1 << 16) * 4 * 8, n


def test_batched_rounds_slices(H, graph):
    g, G = graph
    pats = P.random_patterns(16, seed=9, kmin=3, kmax=6)
    plans = [H.plan(G, p["k"], p["edges"]) for p in pats]
    for mode in (H.SLICE_MIX, H.SLICE_STRIDE):
        for s in (0, 3):
            print("batched rounds slice mode=%d s=%d" % (mode, s), flush=True)
            outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, slice_count=5, slice_id=s, slice_vertex=-1,
                                 slice_mode=mode)
            for p, pl, r in zip(pats, plans, outs):
                o = pl.info()["order"]
                ref = oracle_run(g, p["k"], p["edges"], order=o, slice_count=5, slice_id=s, slice_vertex=o[0],
                                 slice_mode=mode)
                assert cmp_key(r, p["k"]) == cmp_key(ref, p["k"]), (p, mode, s)
                assert r["level_counts"][:p["k"]] == ref["level_counts"][:p["k"]]


def test_batched_rounds_tuned_table_and_no_hash(H, hubs):
    g, G = hubs
    names = ["diamond", "house", "4-clique", "5-clique"]
    plans = [H.plan(G, *P.NAMED[n]) for n in names]
    t = H.autotune(G, plans, slice_count=8, slice_id=7, slice_vertex=-1)
    outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, tune=t)
    nh = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, tune=t, hash=False)
    for n, pl, r, q in zip(names, plans, outs, nh):
        k = P.NAMED[n][0]
        single = H.count(G, pl)
        assert cmp_key(r, k) == cmp_key(single, k), n
        assert q["count"] == single["count"] and q["hash_sum"] == 0


def _table(H, search_j, strat):
    """A tune table: Ext sizes in search_j take `strat` (0 or 1), the others the
    block-cached long lane merge, in every bucket."""
    nb = H.TUNE_BUCKETS
    return H.TuneTable.from_dict({
        "strategy": [[strat if j in search_j else 6 for _ in range(nb)] for j in range(H.KMAX + 1)],
        "chunk_rows": [0] * (H.KMAX + 1), "ms": [[0.0] * nb for _ in range(H.KMAX + 1)],
        "items": [[1] * nb for _ in range(H.KMAX + 1)]})


@pytest.mark.parametrize("search_j,strat", [((1, 3), 0), ((2,), 1), ((1, 2, 3, 4), 0), ((), 0)])
def test_batched_rounds_search_and_merge_launches(H, hubs, search_j, strat):
    """A table that sends some Ext sizes to binary-search or wave-staged strategies
    and the others to lane merges: each query level runs its kind of tile inside
    the level's one extend launch (binary search for both search strategies),
    both kinds share the rounds, and every result equals the query's single run."""
    g, G = hubs
    names = ["triangle", "4-cycle", "diamond", "house", "5-cycle", "4-clique", "tailed-triangle", "5-clique"]
    plans = [H.plan(G, *P.NAMED[n]) for n in names]
    print("batched rounds search j=%s strategy=%d" % (search_j, strat), flush=True)
    t = _table(H, search_j, strat)
    for cap in (0, 1 << 24):
        outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, tune=t, cap=cap)
        for n, pl, r in zip(names, plans, outs):
            k = P.NAMED[n][0]
            single = H.count(G, pl)
            assert cmp_key(r, k) == cmp_key(single, k), (n, cap)
            assert r["level_counts"][:k] == single["level_counts"][:k], (n, cap)
            assert r["level_work"][:k] == single["level_work"][:k], (n, cap)
    nh = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, tune=t, hash=False)
    for n, pl, r in zip(names, plans, nh):
        assert r["count"] == H.count(G, pl)["count"] and r["hash_sum"] == 0, n


def test_batched_rounds_workspace_reuse_and_replays(H, graph):
    """A caller workspace reused across calls of different batches gives the same
    results as fresh allocations, with eager work and synchronisations between."""
    import torch

    g, G = graph
    ws = H.Workspace()
    pa = P.random_patterns(12, seed=10, kmin=3, kmax=6)
    pb = P.random_patterns(5, seed=11, kmin=4, kmax=5)
    plans_a = [H.plan(G, p["k"], p["edges"]) for p in pa]
    plans_b = [H.plan(G, p["k"], p["edges"]) for p in pb]
    want_a = [cmp_key(r, 0) for r in H.count_batch(G, plans_a, engine=H.ENGINE_GRAPH)]
    want_b = [cmp_key(r, 0) for r in H.count_batch(G, plans_b, engine=H.ENGINE_GRAPH)]
    for it in range(3):
        x = torch.arange(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        got_a = [cmp_key(r, 0) for r in H.count_batch(G, plans_a, engine=H.ENGINE_GRAPH, workspace=ws)]
        got_b = [cmp_key(r, 0) for r in H.count_batch(G, plans_b, engine=H.ENGINE_GRAPH, workspace=ws)]
        assert got_a == want_a and got_b == want_b, it
        assert int(x) == (1 << 16) * ((1 << 16) - 1) // 2


def test_batched_rounds_edge_cases_and_errors(H):
    e = gg.from_edges(50, [])
    G = H.load(e.row_ptr, e.col)
    plans = [H.plan(G, *P.NAMED[n]) for n in ["edge", "triangle", "house"]]
    outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH)
    assert [r["count"] for r in outs] == [0, 0, 0]
    k7 = gg.complete(9)
    G7 = H.load(k7.row_ptr, k7.col)
    pl = [H.plan(G7, 7, [(a, b) for a in range(7) for b in range(a + 1, 7)]),
          H.plan(G7, *P.NAMED["6-cycle"])]
    r = H.count_batch(G7, pl, engine=H.ENGINE_GRAPH)
    assert r[0]["count"] == 36  # C(9, 7)
    assert r[1]["count"] == 84 * 60  # C(9, 6) * 6! / 12
    r0 = H.count_batch(G7, pl, engine=H.ENGINE_GRAPH, strategy=0)
    assert [cmp_key(x, 0) for x in r0] == [cmp_key(x, 0) for x in r]
    with pytest.raises(H.HugeError):
        H.count_batch(G7, pl, engine=H.ENGINE_GRAPH, work_limit=10)
