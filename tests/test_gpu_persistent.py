"""GPU parity of the persistent engine (per-workgroup Algorithm 5 with work
stealing) and of batched multi-query launches, against the oracle."""
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import assert_parity, cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu

PERSIST = 2
KMAX = 4  # largest query the persistent kernel is built for

# A persistent-kernel variant for queries of 5 or more vertices hung on the
# house query (k=5, stealing on) and the cause was not found; that variant is
# switched off (the library rejects k > 4 on this engine) and these cases stay
# skipped until it is rebuilt and shown correct.
K5_OFF = "persistent engine is off for k >= 5 (a variant hung on house, cause not found)"


def _k5(name):
    k = P.NAMED[name][0]
    return pytest.param(name, marks=pytest.mark.skip(reason=K5_OFF)) if k > KMAX else name


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def small(H):
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    return g, H.load(g.row_ptr, g.col)


@pytest.mark.parametrize("steal", [1, 0])
@pytest.mark.parametrize("name", [_k5(n) for n in ["triangle", "4-cycle", "diamond", "4-clique", "house", "5-clique",
                                                   "tailed-triangle", "5-cycle", "6-cycle", "3-star", "4-path"]])
def test_persistent_named(H, small, name, steal):
    g, G = small
    k, e = P.NAMED[name]
    r, ref = assert_parity(H, G, g, k, e, engine=PERSIST, work_stealing=steal)
    assert r["count"] > 0


def test_persistent_rejects_large_queries(H, small):
    _, G = small
    k, e = P.NAMED["house"]
    with pytest.raises(RuntimeError, match="persistent engine supports"):
        H.count(G, H.plan(G, k, e), engine=PERSIST)


@pytest.mark.parametrize("name", [_k5(n) for n in ["house", "5-clique", "4-cycle", "diamond", "4-clique"]])
def test_persistent_small_frontier(H, small, name):
    """A small frontier budget keeps per-workgroup levels short, so rows move between workgroups."""
    g, G = small
    k, e = P.NAMED[name]
    assert_parity(H, G, g, k, e, engine=PERSIST, cap=0)


def test_persistent_small_frontier_skewed(H):
    big = gg.rmat(12, 16, seed=4)
    Gb = H.load(big.row_ptr, big.col)
    for name in ["4-cycle", "diamond"]:
        k, e = P.NAMED[name]
        p = H.plan(Gb, k, e)
        a = H.count(Gb, p, engine=PERSIST, cap=0)
        b = H.count(Gb, p)
        assert cmp_key(a, k) == cmp_key(b, k)
        assert a["level_counts"][:k] == b["level_counts"][:k]


@pytest.mark.parametrize("name", [_k5("house"), "4-cycle", "diamond"])
def test_persistent_slices(H, small, name):
    g, G = small
    k, e = P.NAMED[name]
    for s in range(3):
        assert_parity(H, G, g, k, e, engine=PERSIST, slice_count=3, slice_id=s, slice_vertex=1)


@pytest.mark.parametrize("kmax", [4, 5])
def test_batched_patterns_match_single_runs(H, kmax):
    """Queries of 3..4 vertices share one persistent launch; larger ones run on the level engine."""
    g = gg.chung_lu(2000, 8, 2.5, seed=33)
    G = H.load(g.row_ptr, g.col)
    pats = P.random_patterns(16, seed=3, kmin=3, kmax=kmax)
    plans = [H.plan(G, p["k"], p["edges"]) for p in pats]
    outs = H.count_batch(G, plans, engine=PERSIST)
    for p, pl, r in zip(pats, plans, outs):
        ref = oracle_run(g, p["k"], p["edges"], order=pl.info()["order"])
        assert cmp_key(r, p["k"]) == cmp_key(ref, p["k"]), p
        assert r["level_counts"][:p["k"]] == ref["level_counts"][:p["k"]], p


def test_workgroup_balance_with_and_without_stealing(H):
    """Section 7.3's load-balance measure: the standard deviation of per-workgroup
    busy time.  Both runs give the same results; the launch reports its workgroups
    and the mean and spread of their busy times (stealing shrinks the spread on a
    skewed graph)."""
    big = gg.rmat(13, 16, seed=4)
    G = H.load(big.row_ptr, big.col)
    k, e = P.NAMED["diamond"]
    p = H.plan(G, k, e)
    on = H.count(G, p, engine=PERSIST, work_stealing=1)
    off = H.count(G, p, engine=PERSIST, work_stealing=0)
    assert cmp_key(on, k) == cmp_key(off, k)
    for r in (on, off):
        assert r["workgroups"] > 0 and r["wg_busy_ms_mean"] > 0 and r["wg_busy_ms_std"] >= 0
    print("busy ms mean/std: stealing %.3f/%.3f, none %.3f/%.3f" % (
        on["wg_busy_ms_mean"], on["wg_busy_ms_std"], off["wg_busy_ms_mean"], off["wg_busy_ms_std"]))
    assert on["wg_busy_ms_std"] <= off["wg_busy_ms_std"]


def test_persistent_uses_the_caller_workspace(H, small):
    import torch

    g, G = small
    k, e = P.NAMED["4-clique"]
    p = H.plan(G, k, e)
    o = H.exec_opts(engine=PERSIST)
    need = H.workspace_size(G, p, o)
    assert need > 0
    ws = H.Workspace()
    a = H.count(G, p, engine=PERSIST, workspace=ws)
    assert ws.buf is not None and ws.buf.numel() >= need
    b = H.count(G, p, engine=PERSIST, workspace=None)
    assert cmp_key(a, k) == cmp_key(b, k)
