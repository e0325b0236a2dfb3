"""The graph engine: Algorithm 5 with its scheduler on the device, one round of
fixed launches recorded in a hipGraph and replayed until the device says the
query is done.  Its results must equal the oracle's and the level engine's bit
for bit, for every cap, segment size, slice and strategy it runs; replays of the
same query, with eager runs in between, must agree every time."""
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import assert_parity, cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu

GRAPH = 3


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def small(H):
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    return g, H.load(g.row_ptr, g.col)


@pytest.fixture(scope="module")
def hubby(H):
    g = gg.rmat(12, 16, seed=4)
    return g, H.load(g.row_ptr, g.col)


@pytest.mark.parametrize("name", ["triangle", "4-cycle", "diamond", "4-clique", "house", "5-clique", "6-cycle",
                                  "tailed-triangle", "4-path", "edge"])
def test_named_patterns_match_oracle(H, small, name):
    g, G = small
    k, e = P.NAMED[name]
    assert_parity(H, G, g, k, e, engine=GRAPH)


@pytest.mark.parametrize("strategy", [-1, 0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("cap,chunk", [(0, 0), (1 << 20, 300), (4 << 30, 4096), (4 << 30, 0)])
def test_caps_chunks_strategies(H, small, cap, chunk, strategy):
    g, G = small
    for name in ["4-clique", "house", "4-cycle"]:
        k, e = P.NAMED[name]
        assert_parity(H, G, g, k, e, engine=GRAPH, cap=cap, chunk_rows=chunk, strategy=strategy)


def test_slices_and_no_hash(H, small):
    g, G = small
    k, e = P.NAMED["house"]
    p = H.plan(G, k, e)
    order = p.info()["order"]
    for s in range(3):
        r = H.count(G, p, engine=GRAPH, slice_count=3, slice_id=s, slice_vertex=-1)
        ref = oracle_run(g, k, e, order=order, slice_count=3, slice_id=s, slice_vertex=order[0])
        assert cmp_key(r, k) == cmp_key(ref, k), s
        assert r["level_counts"][:k] == ref["level_counts"][:k], s
        r = H.count(G, p, engine=GRAPH, slice_count=3, slice_id=s, slice_vertex=-2)
        ref = oracle_run(g, k, e, order=order, slice_count=3, slice_id=s, slice_pair=(order[0], order[1]))
        assert cmp_key(r, k) == cmp_key(ref, k), s
    r = H.count(G, p, engine=GRAPH, hash=False)
    assert r["count"] == oracle_run(g, k, e, order=order)["count"] and r["hash_sum"] == 0


def test_same_as_level_engine_on_hub_graph(H, hubby):
    g, G = hubby
    for name in ["4-clique", "diamond", "4-cycle", "tailed-triangle"]:
        k, e = P.NAMED[name]
        p = H.plan(G, k, e)
        ref = H.count(G, p, engine=1)
        for cap in (0, 4 << 30):
            r = H.count(G, p, engine=GRAPH, cap=cap)
            assert cmp_key(r, k) == cmp_key(ref, k), (name, cap)
            assert r["level_counts"][:k] == ref["level_counts"][:k], (name, cap)
            assert r["level_work"] == ref["level_work"], (name, cap)


def test_replays_agree_with_eager_runs_in_between(H, hubby):
    """Each count records its round and replays it many times; repeat that with
    eager level-engine runs and synchronisations between the graph runs."""
    import torch

    g, G = hubby
    k, e = P.NAMED["diamond"]
    p = H.plan(G, k, e)
    ref = H.count(G, p, engine=1)
    for i in range(4):
        r = H.count(G, p, engine=GRAPH, cap=0 if i % 2 else 1 << 22, chunk_rows=2000)
        assert r["launches"] > 1
        assert cmp_key(r, k) == cmp_key(ref, k), i
        torch.cuda.synchronize()
        assert cmp_key(H.count(G, p, engine=1, cap=0), k) == cmp_key(ref, k)


def test_batch_on_graph_engine(H, small):
    g, G = small
    names = ["triangle", "diamond", "house", "5-clique", "edge"]
    plans = [H.plan(G, *P.NAMED[n]) for n in names]
    outs = H.count_batch(G, plans, engine=GRAPH)
    for n, pl, r in zip(names, plans, outs):
        assert cmp_key(r, pl.k) == cmp_key(H.count(G, pl, engine=1), pl.k), n


def test_edgeless_and_errors(H):
    import numpy as np

    rp = np.zeros(9, np.int64)
    col = np.zeros(0, np.int32)
    G0 = H.load(rp, col)
    k, e = P.NAMED["triangle"]
    assert H.count(G0, H.plan(G0, k, e), engine=GRAPH)["count"] == 0
    g = gg.chung_lu(500, 6, 2.5, seed=2)
    G = H.load(g.row_ptr, g.col)
    p = H.plan(G, *P.NAMED["diamond"])
    for bad in [dict(work_limit=10)]:
        with pytest.raises(H.HugeError) as ei:
            H.count(G, p, engine=GRAPH, **bad)
        assert ei.value.name == "HUGE_EINVAL", bad
    with pytest.raises(H.HugeError) as ei:
        H.enumerate_matches(G, p, buf_rows=100, engine=GRAPH)
    assert ei.value.name == "HUGE_EINVAL"


def _table(H, seed):
    import random

    rng = random.Random(seed)
    t = H.TuneTable()
    for j in range(H.KMAX + 1):
        t.chunk_rows[j] = rng.choice([0, 300, 4096, 1 << 20])
        for c in range(H.TUNE_BUCKETS):
            t.strategy[j][c] = rng.choice([-1] + list(range(H.STRAT_COUNT)))
    return t


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tuned_dispatch_matches_level_engine_and_oracle(H, small, hubby, seed):
    """Per-bucket dispatch inside the recorded round: every strategy, random
    segment sizes, both frontier extremes."""
    t = _table(H, seed)
    g, G = small
    for name in ["4-clique", "house", "diamond"]:
        k, e = P.NAMED[name]
        assert_parity(H, G, g, k, e, engine=GRAPH, tune=t)
        assert_parity(H, G, g, k, e, engine=GRAPH, tune=t, cap=0, slice_count=3, slice_id=1, slice_vertex=2)
    g2, G2 = hubby
    for name in ["4-clique", "4-cycle", "tailed-triangle"]:
        k, e = P.NAMED[name]
        p = H.plan(G2, k, e)
        ref = H.count(G2, p, engine=1, tune=t)
        r = H.count(G2, p, engine=GRAPH, tune=t)
        assert cmp_key(r, k) == cmp_key(ref, k), name
        assert r["level_counts"][:k] == ref["level_counts"][:k] and r["level_work"] == ref["level_work"], name


def test_autotuned_table_on_graph_engine(H, hubby):
    g, G = hubby
    plans = [H.plan(G, *P.NAMED[n]) for n in ["diamond", "4-clique"]]
    t = H.autotune(G, plans, slice_count=4, slice_id=0)
    for p in plans:
        ref = H.count(G, p, engine=1, tune=t)
        for _ in range(2):
            assert cmp_key(H.count(G, p, engine=GRAPH, tune=t), p.k) == cmp_key(ref, p.k)
