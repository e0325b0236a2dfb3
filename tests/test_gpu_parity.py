"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the
same seeded inputs.  Counts, set-hash sum and xor, and per-prefix level
counts must be bit-identical."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from graphgen import patterns as P
from tests.gpu_common import assert_parity, cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu

TRI = P.NAMED["triangle"]
C4 = P.NAMED["4-cycle"]


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def c1(H):
    """Chung-Lu n=16384, mean degree 16, exponent 2.5, exact pairwise draws, seed 1."""
    g = gg.chung_lu(16384, 16, 2.5, seed=1, exact=True)
    return g, H.load(g.row_ptr, g.col)


@pytest.fixture(scope="module")
def small(H):
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    return g, H.load(g.row_ptr, g.col)


def test_relabel_is_degree_rank(H, c1):
    g, G = c1
    rp, col, inv = G.export()
    rank = oracle.ranks(g.row_ptr)
    assert np.array_equal(inv[rank], np.arange(g.n, dtype=np.int32))
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a, b = rank[src].astype(np.int64), rank[g.col].astype(np.int64)
    order = np.lexsort((b, a))
    want_col = b[order].astype(np.int32)
    want_rp = np.concatenate([[0], np.cumsum(np.bincount(a, minlength=g.n))]).astype(np.int64)
    assert np.array_equal(rp, want_rp)
    assert np.array_equal(col, want_col)
    info = G.info()
    d = np.diff(g.row_ptr).astype(np.float64)
    assert info["max_degree"] == int(d.max())
    for p in range(8):
        assert info["degree_moments"][p] == pytest.approx(float((d ** p).sum()), rel=1e-12)


def test_device_pointer_load_matches_host_load(H, small):
    import torch

    g, G = small
    Gd = H.load(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda())
    a, b = G.export(), Gd.export()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name", ["triangle", "4-cycle"])
def test_c1_full_parity(H, c1, name):
    g, G = c1
    k, e = P.NAMED[name]
    r, ref = assert_parity(H, G, g, k, e)
    assert r["count"] > 0


@pytest.mark.parametrize("name", sorted(P.NAMED))
def test_named_patterns(H, small, name):
    g, G = small
    k, e = P.NAMED[name]
    assert_parity(H, G, g, k, e)


def test_random_patterns(H):
    g = gg.chung_lu(2000, 8, 2.5, seed=33)
    G = H.load(g.row_ptr, g.col)
    for pat in P.random_patterns(24, seed=7, kmin=3, kmax=6):
        assert_parity(H, G, g, pat["k"], pat["edges"])


def test_every_order_gives_the_same_matches(H):
    g = gg.chung_lu(1500, 9, 2.4, seed=4)
    G = H.load(g.row_ptr, g.col)
    for name in ["house", "diamond", "tailed-triangle"]:
        k, e = P.NAMED[name]
        ref = oracle_run(g, k, e)
        adj = {frozenset(x) for x in e}
        seen = 0
        for order in itertools.permutations(range(k)):
            if any(not any(frozenset((order[p], order[i])) in adj for p in range(i)) for i in range(1, k)):
                continue
            r, _ = assert_parity(H, G, g, k, e, order=order)
            assert cmp_key(r, k) == cmp_key(ref, k)
            seen += 1
        assert seen >= 4


@pytest.mark.parametrize("name", ["triangle", "4-cycle", "house"])
def test_root_slices(H, c1, name):
    g, G = c1
    k, e = P.NAMED[name]
    full = H.count(G, H.plan(G, k, e))
    S = 8
    cs, hs, hx = 0, 0, 0
    for s in range(S):
        r, _ = assert_parity(H, G, g, k, e, slice_count=S, slice_id=s)
        cs += r["count"]
        hs = (hs + r["hash_sum"]) & ((1 << 64) - 1)
        hx ^= r["hash_xor"]
    assert (cs, hs, hx) == (full["count"], full["hash_sum"], full["hash_xor"])


@pytest.mark.parametrize("cap", [0, 1 << 20, 64 << 20, float("inf")])
@pytest.mark.parametrize("chunk", [0, 777])
def test_bounded_frontier_same_results(H, small, cap, chunk):
    g, G = small
    for name in ["5-clique", "house", "4-cycle"]:
        k, e = P.NAMED[name]
        r, ref = assert_parity(H, G, g, k, e, cap=cap, chunk_rows=chunk)
        if cap not in (0, float("inf")):
            assert r["peak_frontier_bytes"] <= cap


def test_zero_cap_is_depth_first_and_bounded(H, small):
    g, G = small
    k, e = P.NAMED["house"]
    r = H.count(G, H.plan(G, k, e), cap=0)
    big = H.count(G, H.plan(G, k, e), cap=float("inf"))
    assert cmp_key(r, k) == cmp_key(big, k)
    # smallest workable queues: 4096 rows per materialised level
    assert r["peak_frontier_bytes"] <= 4096 * 4 * (3 + 4)
    assert r["launches"] > big["launches"]


def test_rmat_hubs(H):
    g = gg.rmat(13, 16, seed=9)
    G = H.load(g.row_ptr, g.col)
    for name in ["4-clique", "diamond", "4-cycle", "triangle"]:
        k, e = P.NAMED[name]
        assert_parity(H, G, g, k, e)


def test_edge_query(H, small):
    g, G = small
    k, e = P.NAMED["edge"]
    r, ref = assert_parity(H, G, g, k, e)
    assert r["count"] == g.m
    rows = H.enumerate_matches(G, H.plan(G, k, e), buf_rows=1000)["rows"]
    assert rows.shape == (g.m, 2)
    got = {frozenset(map(int, x)) for x in rows}
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    want = {frozenset((int(a), int(b))) for a, b in zip(src, g.col)}
    assert got == want


@pytest.fixture(scope="module")
def tiny(H):
    g = gg.chung_lu(700, 6, 2.5, seed=5)
    return g, H.load(g.row_ptr, g.col)


@pytest.mark.parametrize("name", ["triangle", "4-cycle", "house", "tailed-triangle"])
def test_enumerate_rows(H, tiny, name):
    g, G = tiny
    k, e = P.NAMED[name]
    p = H.plan(G, k, e)
    out = H.enumerate_matches(G, p, buf_rows=4096)
    rows = out["rows"]
    ref = oracle_run(g, k, e)
    assert rows.shape[0] == ref["count"] == out["count"]
    # every row is a match of q (query-vertex order, original IDs) ...
    adj = set(zip(np.repeat(np.arange(g.n), np.diff(g.row_ptr)).tolist(), g.col.tolist()))
    rank = oracle.ranks(g.row_ptr)
    for a, b in e:
        assert all((int(x), int(y)) in adj for x, y in zip(rows[:, a], rows[:, b]))
    for a, b in p.info()["sb_pairs"]:
        assert np.all(rank[rows[:, a]] < rank[rows[:, b]])
    assert all(len(set(r.tolist())) == k for r in rows)
    # ... and the rows are the oracle's subgraphs: same set-hash sum and xor
    hs, hx = 0, 0
    for r in rows:
        h = oracle.set_hash([(int(r[a]), int(r[b])) for a, b in e], rank)
        hs = (hs + h) & ((1 << 64) - 1)
        hx ^= h
    assert (hs, hx) == (ref["hash_sum"], ref["hash_xor"])
    assert len({tuple(sorted(map(int, r))) + tuple(sorted(tuple(sorted((int(r[a]), int(r[b])))) for a, b in e)) for r in rows}) == rows.shape[0]


def test_enumerate_stop(H, tiny):
    g, G = tiny
    k, e = P.NAMED["triangle"]
    calls = []

    def cb(rows):
        calls.append(rows.shape[0])
        return True

    out = H.enumerate_matches(G, H.plan(G, k, e), buf_rows=100, callback=cb)
    assert out["stopped"] and len(calls) == 1 and out["count"] == calls[0] <= 100


@pytest.mark.parametrize("defect", ["unsorted", "duplicate", "self", "range", "asym", "rowptr"])
def test_bad_graphs_rejected(H, defect):
    g = gg.gnp(50, 0.2, seed=2)
    rp, col = g.row_ptr.copy(), g.col.copy()
    u = int(np.argmax(np.diff(rp)))
    a = int(rp[u])
    if defect == "unsorted":
        col[a], col[a + 1] = col[a + 1], col[a]
    elif defect == "duplicate":
        col[a + 1] = col[a]
    elif defect == "self":
        col[a] = u
        col[a:rp[u + 1]] = np.sort(col[a:rp[u + 1]])
    elif defect == "range":
        col[rp[u + 1] - 1] = 50
    elif defect == "asym":
        e = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)])
        rp, col = e.row_ptr.copy(), e.col.copy()
        col[0] = 2
    elif defect == "rowptr":
        rp[3] = rp[4] + 1
    with pytest.raises(H.HugeError) as ei:
        H.load(rp, col)
    assert ei.value.name == "HUGE_EGRAPH", str(ei.value)


@pytest.mark.parametrize("strategy", [0, 1, 2, 3, 4, 5, 6])
def test_strategies_agree(H, small, strategy):
    g, G = small
    for name in ["4-clique", "diamond", "4-cycle", "house", "5-clique"]:
        k, e = P.NAMED[name]
        assert_parity(H, G, g, k, e, strategy=strategy)
    g2 = gg.chung_lu(2000, 8, 2.5, seed=33)
    G2 = H.load(g2.row_ptr, g2.col)
    for pat in P.random_patterns(6, seed=strategy + 40, kmin=4, kmax=5):
        assert_parity(H, G2, g2, pat["k"], pat["edges"], strategy=strategy, chunk_rows=5000)
    g3 = gg.rmat(10, 8, seed=17)
    G3 = H.load(g3.row_ptr, g3.col)
    for name in ["4-clique", "diamond", "4-cycle"]:
        k, e = P.NAMED[name]
        assert_parity(H, G3, g3, k, e, strategy=strategy)
    # a graph whose 12 vertices of degree >= 256 answer membership from their bitmaps,
    # next to lists searched in memory
    g4 = gg.rmat(11, 16, seed=9)
    G4 = H.load(g4.row_ptr, g4.col)
    assert G4.info()["hub_count"] > 0
    for name in ["4-clique", "diamond"]:
        k, e = P.NAMED[name]
        assert_parity(H, G4, g4, k, e, strategy=strategy)
    k, e = P.NAMED["5-clique"]
    assert_parity(H, G4, g4, k, e, strategy=strategy, slice_count=16, slice_id=3, slice_vertex=0)


@pytest.mark.parametrize("sv", [1, 3, 4])
def test_slice_on_other_vertex(H, small, sv):
    g, G = small
    k, e = P.NAMED["house"]
    full = H.count(G, H.plan(G, k, e))
    cs = 0
    for s in range(4):
        r, _ = assert_parity(H, G, g, k, e, slice_count=4, slice_id=s, slice_vertex=sv)
        cs += r["count"]
    assert cs == full["count"]


def test_hub_bitmaps_do_not_change_results(H, monkeypatch):
    g = gg.rmat(13, 16, seed=9)
    base = H.load(g.row_ptr, g.col, hub_bitmaps=False)
    assert base.info()["hub_count"] == 0
    full = H.load(g.row_ptr, g.col)
    assert full.info()["hub_count"] > 0 and full.info()["hub_min_degree"] >= 256
    words = (g.n + 31) // 32
    monkeypatch.setenv("HUGE_HUB_BYTES", str(3 * 4 * words))
    part = H.load(g.row_ptr, g.col)
    assert part.info()["hub_count"] == 3
    for name in ["4-clique", "diamond", "4-cycle", "triangle"]:
        k, e = P.NAMED[name]
        ref = H.count(base, H.plan(base, k, e))
        for G in (full, part):
            for strategy in (0, 1, 2, 5, 6):
                r = H.count(G, H.plan(G, k, e), strategy=strategy)
                assert cmp_key(r, k) == cmp_key(ref, k), (name, strategy)


def test_count_without_hash(H, small):
    g, G = small
    for name in ["triangle", "4-cycle", "house"]:
        k, e = P.NAMED[name]
        p = H.plan(G, k, e)
        ref = oracle_run(g, k, e, order=p.info()["order"])
        for strategy in (0, 1, 2, 5, 6):
            r = H.count(G, p, hash=False, strategy=strategy)
            assert r["count"] == ref["count"] and r["hash_sum"] == 0 and r["hash_xor"] == 0
            assert r["level_counts"][:k] == ref["level_counts"][:k]
