"""Per-bucket dispatch and the autotuner: results never depend on the table;
prefix plans and work limits behave as documented."""
import json
import random

import numpy as np
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import assert_parity, cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def hubby(H):
    g = gg.rmat(12, 16, seed=4)
    return g, H.load(g.row_ptr, g.col)


def _random_table(H, seed, k=4):
    # Small segments cost one host synchronisation each: on queries of 5 or
    # more vertices a level holds ~10^8 rows here, so those draw >= 2^16.
    rng = random.Random(seed)
    t = H.TuneTable()
    sizes = [0, 300, 4096, 1 << 20] if k <= 4 else [0, 1 << 16, 1 << 18, 1 << 20]
    for j in range(H.KMAX + 1):
        t.chunk_rows[j] = rng.choice(sizes)
        for c in range(H.TUNE_BUCKETS):
            t.strategy[j][c] = rng.choice([-1] + list(range(H.STRAT_COUNT)))
    return t


@pytest.mark.parametrize("name", ["triangle", "4-cycle", "diamond", "4-clique", "house", "5-clique", "tailed-triangle"])
def test_random_tables_do_not_change_results(H, hubby, name):
    g, G = hubby
    k, e = P.NAMED[name]
    p = H.plan(G, k, e)
    ref = H.count(G, p)
    # depth-first runs (cap 0: 4096-row queues) of the 5-vertex queries take
    # ~770K launches here; they get a 1 MiB frontier instead
    caps = [4 << 30, 0] if k <= 4 else [4 << 30, 1 << 20]
    for seed in range(3):
        t = _random_table(H, seed * 7 + k, k)
        for cap in caps:
            r = H.count(G, p, tune=t, cap=cap)
            assert cmp_key(r, k) == cmp_key(ref, k), (seed, cap)
            assert r["level_counts"][:k] == ref["level_counts"][:k]


def test_table_parity_with_oracle_and_slices(H):
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    t = _random_table(H, 99)
    for name in ["house", "4-cycle", "diamond"]:
        k, e = P.NAMED[name]
        assert_parity(H, G, g, k, e, tune=t)
        assert_parity(H, G, g, k, e, tune=t, slice_count=4, slice_id=1, slice_vertex=2)


def test_table_enumerate_rows(H):
    g = gg.chung_lu(700, 6, 2.5, seed=5)
    G = H.load(g.row_ptr, g.col)
    t = _random_table(H, 5)
    k, e = P.NAMED["house"]
    p = H.plan(G, k, e)
    a, b = [], []
    H.enumerate_matches(G, p, buf_rows=1000, callback=lambda rows: a.extend(map(tuple, rows.tolist())))
    H.enumerate_matches(G, p, buf_rows=1000, callback=lambda rows: b.extend(map(tuple, rows.tolist())), tune=t)
    assert len(a) == len(set(a)) > 0
    assert sorted(a) == sorted(b)


def test_autotune_table_and_cache(H, hubby, tmp_path):
    g, G = hubby
    plans = [H.plan(G, *P.NAMED[n]) for n in ["4-cycle", "diamond", "house"]]
    cache = str(tmp_path / "tune.json")
    t = H.autotune(G, plans, cache=cache, slice_count=4, slice_id=0)
    seen = [(j, c) for j in range(H.KMAX + 1) for c in range(H.TUNE_BUCKETS) if t.items[j][c] > 0]
    assert seen, "the sample did no intersection work"
    for j, c in seen:
        assert 0 <= t.strategy[j][c] < H.STRAT_COUNT
        assert t.ms[j][c] > 0
    for j in range(H.KMAX + 1):
        if any(t.items[j][c] for c in range(H.TUNE_BUCKETS)):
            assert t.chunk_rows[j] in (1 << 18, 1 << 20, 1 << 22)
    with open(cache) as f:
        d = json.load(f)
    assert len(d) == 1 and list(d.values())[0]["strategy"] == t.to_dict()["strategy"]
    t2 = H.autotune(G, plans, cache=cache, slice_count=4, slice_id=0)  # served from the cache
    assert t2.to_dict() == t.to_dict()
    for p, name in zip(plans, ["4-cycle", "diamond", "house"]):
        k, e = P.NAMED[name]
        assert cmp_key(H.count(G, p, tune=t), k) == cmp_key(oracle_run(g, k, e), k)


@pytest.mark.parametrize("name", ["house", "5-clique", "diamond", "6-cycle"])
def test_prefix_plan_counts_are_level_counts(H, name):
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    k, e = P.NAMED[name]
    p = H.plan(G, k, e)
    full = H.count(G, p)
    ref = oracle_run(g, k, e, order=p.info()["order"])
    assert full["level_counts"][:k] == ref["level_counts"][:k]
    for s in range(2, k + 1):
        q = H.plan_prefix(p, s)
        assert q.info()["order"] == list(range(s))
        r = H.count(G, q)
        assert r["count"] == full["level_counts"][s - 1], s
        assert r["level_counts"][:s] == full["level_counts"][:s]
    with pytest.raises(RuntimeError):
        H.plan_prefix(p, 1)


def test_work_limit_stops(H, hubby):
    g, G = hubby
    k, e = P.NAMED["4-cycle"]
    p = H.plan(G, k, e)
    full = H.count(G, p)
    assert not full["stopped"]
    r = H.count(G, p, work_limit=1000, chunk_rows=4096)
    assert r["stopped"] and r["count"] < full["count"]
    r = H.count(G, p, work_limit=1 << 62)
    assert not r["stopped"] and cmp_key(r, k) == cmp_key(full, k)


@pytest.mark.parametrize("name", ["house", "diamond", "4-clique", "6-cycle"])
def test_edge_slices_match_oracle_and_partition(H, name):
    """slice_vertex=-2 keeps the matches whose first two matched vertices' ordered
    rank pair hashes into the slice; the slices partition the matches."""
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    k, e = P.NAMED[name]
    p = H.plan(G, k, e)
    order = p.info()["order"]
    full = H.count(G, p)
    cs, hs, hx = 0, 0, 0
    for s in range(5):
        r = H.count(G, p, slice_count=5, slice_id=s, slice_vertex=-2)
        ref = oracle_run(g, k, e, order=order, slice_count=5, slice_id=s, slice_pair=(order[0], order[1]))
        assert cmp_key(r, k) == cmp_key(ref, k), s
        assert r["level_counts"][1:k] == ref["level_counts"][1:k], s
        cs += r["count"]
        hs = (hs + r["hash_sum"]) % (1 << 64)
        hx ^= r["hash_xor"]
    assert (cs, hs, hx) == (full["count"], full["hash_sum"], full["hash_xor"])
