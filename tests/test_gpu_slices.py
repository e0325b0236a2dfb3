"""GPU parity of strided root slices and double slices against the oracle.

A strided slice keeps the matches whose first matched vertex has rank
s mod S; the engines read only that slice's edge-array entries (gathered into
the workspace).  A second vertex slice narrows any slice again, so two plans
with different first vertices can run the same sample, each reading only its
own slice's entries."""
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def cl(H):
    g = gg.chung_lu(6000, 14, 2.3, seed=31)
    return g, H.load(g.row_ptr, g.col)


@pytest.fixture(scope="module")
def rm(H):
    g = gg.rmat(11, 16, seed=32)
    return g, H.load(g.row_ptr, g.col)


PATTERNS = ["edge", "wedge", "triangle", "4-cycle", "diamond", "house", "5-clique"]


@pytest.mark.parametrize("name", PATTERNS)
@pytest.mark.parametrize("engine", ["levels", "graph"])
def test_strided_root_slices(H, cl, name, engine):
    g, G = cl
    k, e = P.NAMED[name]
    p = H.plan(G, k, e)
    order = p.info()["order"]
    eng = H.ENGINE_GRAPH if engine == "graph" else H.ENGINE_LEVELS
    S = 5
    tot = [0, 0, 0]
    for s in range(S):
        print("strided slice %s %s s=%d" % (name, engine, s), flush=True)
        r = H.count(G, p, slice_count=S, slice_id=s, slice_vertex=-1, slice_mode=H.SLICE_STRIDE, engine=eng)
        ref = oracle_run(g, k, e, order=order, slice_count=S, slice_id=s, slice_vertex=order[0], slice_mode=1)
        assert cmp_key(r, k) == cmp_key(ref, k), (name, s, r, ref)
        assert r["level_counts"][1:k] == ref["level_counts"][1:k], (name, s)
        tot = [tot[0] + r["count"], (tot[1] + r["hash_sum"]) % (1 << 64), tot[2] ^ r["hash_xor"]]
    full = H.count(G, p, engine=eng)
    assert tuple(tot) == cmp_key(full, k)


@pytest.mark.parametrize("name", ["triangle", "diamond", "house", "5-cycle"])
def test_strided_slices_rmat_small_segments_and_caps(H, rm, name):
    """Hub-heavy R-MAT: gathered level 2 split over many segments, and small frontier caps."""
    g, G = rm
    k, e = P.NAMED[name]
    p = H.plan(G, k, e)
    order = p.info()["order"]
    for S, s, chunk, cap in [(64, 63, 300, 1 << 20), (29, 3, 0, 0), (1000, 999, 0, 1 << 24)]:
        print("rmat strided %s S=%d s=%d chunk=%d cap=%d" % (name, S, s, chunk, cap), flush=True)
        r = H.count(G, p, slice_count=S, slice_id=s, slice_vertex=-1, slice_mode=H.SLICE_STRIDE,
                    chunk_rows=chunk, cap=cap)
        ref = oracle_run(g, k, e, order=order, slice_count=S, slice_id=s, slice_vertex=order[0], slice_mode=1)
        assert cmp_key(r, k) == cmp_key(ref, k), (name, S, s)
        assert r["level_counts"][:k] == ref["level_counts"][:k]
        if cap:
            assert r["peak_frontier_bytes"] <= cap


@pytest.mark.parametrize("name", ["diamond", "house", "tailed-triangle"])
def test_double_slices_agree_across_orders(H, cl, name):
    """Two orders with different first vertices a, b: order A with (a: s1 of S1) and
    second slice (b: s2 of S2), order B with the roles swapped, select the same
    matches: equal to each other and to the oracle."""
    g, G = cl
    k, e = P.NAMED[name]
    import itertools
    adj = {(a, b) for a, b in e} | {(b, a) for a, b in e}
    orders = [list(o) for o in itertools.permutations(range(k))
              if all(any((o[i], o[j]) in adj for j in range(i)) for i in range(1, k))]
    oa = orders[0]
    ob = next(o for o in orders if o[0] != oa[0])
    pa, pb = H.plan(G, k, e, order=oa), H.plan(G, k, e, order=ob)
    S1, S2 = 3, 4
    for s1, s2 in [(0, 0), (2, 3), (1, 2)]:
        print("double slice %s s1=%d s2=%d" % (name, s1, s2), flush=True)
        ra = H.count(G, pa, slice_count=S1, slice_id=s1, slice_vertex=-1, slice_mode=H.SLICE_STRIDE,
                     slice2=(ob[0], S2, s2))
        rb = H.count(G, pb, slice_count=S2, slice_id=s2, slice_vertex=-1, slice_mode=H.SLICE_STRIDE,
                     slice2=(oa[0], S1, s1), engine=H.ENGINE_GRAPH)
        ref = oracle_run(g, k, e, order=oa, slice_count=S1, slice_id=s1, slice_vertex=oa[0], slice_mode=1,
                         slice2=(ob[0], S2, s2))
        assert cmp_key(ra, k) == cmp_key(ref, k), (name, s1, s2)
        assert cmp_key(rb, k) == cmp_key(ref, k), (name, s1, s2)
        assert ra["level_counts"][1:k] == ref["level_counts"][1:k]


def test_enumerate_strided_slice_rows(H, cl):
    g, G = cl
    k, e = P.NAMED["diamond"]
    p = H.plan(G, k, e)
    order = p.info()["order"]
    d = H.enumerate_matches(G, p, buf_rows=1000, slice_count=9, slice_id=4, slice_vertex=-1,
                            slice_mode=H.SLICE_STRIDE)
    ref = oracle_run(g, k, e, order=order, slice_count=9, slice_id=4, slice_vertex=order[0], slice_mode=1)
    assert d["count"] == ref["count"] == d["rows"].shape[0]
    assert len({tuple(r) for r in d["rows"].tolist()}) == d["count"]


def test_slice_option_errors(H, cl):
    g, G = cl
    k, e = P.NAMED["triangle"]
    p = H.plan(G, k, e)
    bad = [dict(slice2=(0, 0, 3, 1)),
           dict(slice_mode=2),
           dict(slice2=(5, 3, 0)),
           dict(slice2=(1, 3, 3)),
           dict(slice_count=4, slice_id=1, slice_mode=H.SLICE_STRIDE, engine=H.ENGINE_PERSISTENT)]
    for kw in bad:
        with pytest.raises(H.HugeError) as ei:
            H.count(G, p, **kw)
        assert ei.value.name == "HUGE_EINVAL", kw


@pytest.mark.parametrize("name", ["edge", "triangle", "4-cycle", "diamond", "house", "5-clique"])
@pytest.mark.parametrize("engine", ["levels", "graph"])
def test_strided_edge_slices(H, cl, name, engine):
    """Edge slices strided by entry index (every S-th entry of the relabelled CSR
    from s on, read without a scan): the oracle's strided pair slice on the plan's
    first two vertices, and they add up to the whole."""
    g, G = cl
    k, e = P.NAMED[name]
    p = H.plan(G, k, e)
    o = p.info()["order"]
    eng = H.ENGINE_GRAPH if engine == "graph" else H.ENGINE_LEVELS
    S = 7
    tot = [0, 0, 0]
    for s in range(S):
        r = H.count(G, p, slice_count=S, slice_id=s, slice_vertex=-2, slice_mode=H.SLICE_STRIDE, engine=eng)
        ref = oracle_run(g, k, e, order=o, slice_count=S, slice_id=s, slice_pair=(o[0], o[1]), slice_mode=1)
        assert cmp_key(r, k) == cmp_key(ref, k), (name, s)
        assert r["level_counts"][1:k] == ref["level_counts"][1:k], (name, s)
        tot = [tot[0] + r["count"], (tot[1] + r["hash_sum"]) % (1 << 64), tot[2] ^ r["hash_xor"]]
    assert tuple(tot) == cmp_key(H.count(G, p, engine=eng), k)


@pytest.mark.parametrize("name", ["diamond", "house", "tailed-triangle"])
def test_double_edge_slices_agree_across_orders(H, rm, name):
    """Two orders whose first pairs differ: order A on its strided edge slice s1 of
    S1 with a second pair slice on B's first pair (s2 of S2), order B the other way
    round: the same matches, equal to the oracle's, in batches too."""
    import itertools

    g, G = rm
    k, e = P.NAMED[name]
    adj = {(a, b) for a, b in e} | {(b, a) for a, b in e}
    orders = [list(o) for o in itertools.permutations(range(k))
              if all(any((o[i], o[j]) in adj for j in range(i)) for i in range(1, k))]
    oa = orders[0]
    ob = next(o for o in orders if {o[0], o[1]} != {oa[0], oa[1]})
    pa, pb = H.plan(G, k, e, order=oa), H.plan(G, k, e, order=ob)
    for S1, s1, S2, s2 in [(5, 2, 3, 1), (64, 10, 16, 3)]:
        ka = dict(slice_count=S1, slice_id=s1, slice_vertex=-2, slice_mode=H.SLICE_STRIDE, slice2=(ob[0], ob[1], S2, s2))
        kb = dict(slice_count=S2, slice_id=s2, slice_vertex=-2, slice_mode=H.SLICE_STRIDE, slice2=(oa[0], oa[1], S1, s1))
        ra = H.count(G, pa, **ka)
        rb = H.count(G, pb, engine=H.ENGINE_GRAPH, **kb)
        rbb = H.count_batch(G, [pb], engine=H.ENGINE_GRAPH, **kb)[0]
        ref = oracle_run(g, k, e, order=oa, slice_count=S1, slice_id=s1, slice_pair=(oa[0], oa[1]), slice_mode=1,
                         slice2=(ob[0], ob[1], S2, s2))
        assert cmp_key(ra, k) == cmp_key(ref, k) == cmp_key(rb, k) == cmp_key(rbb, k), (name, S1, s1)
        assert ra["level_counts"][1:k] == ref["level_counts"][1:k]


def test_strided_edge_slices_batched_and_enumerated(H, rm):
    g, G = rm
    names = ["triangle", "diamond", "house", "5-cycle", "4-clique"]
    plans = [H.plan(G, *P.NAMED[n]) for n in names]
    outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH, slice_count=50, slice_id=7, slice_vertex=-2,
                         slice_mode=H.SLICE_STRIDE)
    for n, pl, r in zip(names, plans, outs):
        k, e = P.NAMED[n]
        o = pl.info()["order"]
        ref = oracle_run(g, k, e, order=o, slice_count=50, slice_id=7, slice_pair=(o[0], o[1]), slice_mode=1)
        assert cmp_key(r, k) == cmp_key(ref, k), n
    pl = plans[1]
    d = H.enumerate_matches(G, pl, buf_rows=512, slice_count=50, slice_id=7, slice_vertex=-2,
                            slice_mode=H.SLICE_STRIDE)
    assert d["count"] == outs[1]["count"] == d["rows"].shape[0]
