"""Pins of the oracle to things other than itself: published known-answer
vectors, closed-form counts, adjacency-matrix identities, brute force over all
injective maps, and group-theoretic identities of symmetry breaking."""
import itertools
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from graphgen import patterns as P
from tests import closed_forms as cf
from tests.named_graphs import by_name

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_splitmix64_known_answers():
    kat = _golden("kat.json")["splitmix64"]
    for x, y in zip(kat["inputs_hex"], kat["outputs_hex"]):
        assert oracle.mix64(int(x, 16)) == int(y, 16)
    # the inputs are the published generator's successive states
    g = 0x9E3779B97F4A7C15
    assert [int(x, 16) for x in kat["inputs_hex"]] == [(g * i) & M64 for i in range(1, 5)]


def test_philox_known_answers():
    for c in _golden("kat.json")["philox4x32_10"]["cases"]:
        out = gg.philox4x32_10([int(x, 16) for x in c["ctr"]], [int(x, 16) for x in c["key"]])
        assert out == [int(x, 16) for x in c["out"]]


@pytest.mark.parametrize("case", _golden("closed_forms.json")["cases"], ids=lambda c: c["graph"] + ":" + c["pattern"])
def test_closed_form_counts(case):
    g = by_name(case["graph"])
    k, e = P.NAMED[case["pattern"]]
    r = oracle.enumerate_query(g.row_ptr, g.col, k, e)
    assert r["count"] == case["count"], case["why"]
    rc = oracle.enumerate_query(g.row_ptr, g.col, k, e, mode=oracle.MODE_CANON)
    assert (rc["count"], rc["hash_sum"], rc["hash_xor"]) == (r["count"], r["hash_sum"], r["hash_xor"])


def test_automorphism_orders():
    aut = _golden("closed_forms.json")["automorphisms"]
    for name, order in aut.items():
        if name.startswith("_"):
            continue
        k, e = P.NAMED[name]
        A = oracle.automorphisms(k, e)
        assert A.shape[0] == order
        # every listed map is a permutation preserving the edge set
        es = {frozenset(x) for x in e}
        for p in A:
            assert sorted(p.tolist()) == list(range(k))
            assert {frozenset((int(p[a]), int(p[b]))) for a, b in e} == es


def test_grochow_kellis_pairs_of_named_patterns():
    expect = {
        "triangle": [(0, 1), (0, 2), (1, 2)],
        "4-cycle": [(0, 1), (0, 2), (0, 3), (1, 3)],
        "diamond": [(0, 3), (1, 2)],
        "4-clique": [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
        "house": [(0, 1)],
        "5-clique": [(a, b) for a in range(5) for b in range(a + 1, 5)],
    }
    for name, pairs in expect.items():
        k, e = P.NAMED[name]
        assert sorted(oracle.sb_pairs(k, e)) == sorted(pairs), name


def test_sb_identities_on_random_graph():
    """count_SB * |Aut| = number of injective maps, the hash sum over maps is
    |Aut| times the set-hash sum, and SB agrees with the canonical mode."""
    g = gg.gnp(40, 0.3, seed=11)
    for name in ["triangle", "4-cycle", "diamond", "4-clique", "house", "tailed-triangle", "3-star", "5-cycle"]:
        k, e = P.NAMED[name]
        naut = oracle.automorphisms(k, e).shape[0]
        sb = oracle.enumerate_query(g.row_ptr, g.col, k, e)
        al = oracle.enumerate_query(g.row_ptr, g.col, k, e, mode=oracle.MODE_ALL)
        cn = oracle.enumerate_query(g.row_ptr, g.col, k, e, mode=oracle.MODE_CANON)
        assert sb["count"] > 0, name
        assert sb["count"] * naut == al["count"], name
        assert (sb["hash_sum"] * naut) & M64 == al["hash_sum"], name
        assert (cn["count"], cn["hash_sum"], cn["hash_xor"]) == (sb["count"], sb["hash_sum"], sb["hash_xor"]), name


@pytest.mark.parametrize("n,p,seed", [(8, 0.55, 1), (9, 0.45, 2)])
def test_brute_force_all_small_patterns(n, p, seed):
    g = gg.gnp(n, p, seed=seed)
    pats = [(k, e) for k in (2, 3, 4) for e in P.all_connected(k)]
    pats += [(5, e) for e in P.all_connected(5)[::3]]
    for k, e in pats:
        bf = oracle.brute_force(g.row_ptr, g.col, k, e)
        sb = oracle.enumerate_query(g.row_ptr, g.col, k, e)
        al = oracle.enumerate_query(g.row_ptr, g.col, k, e, mode=oracle.MODE_ALL)
        assert (sb["count"], sb["hash_sum"], sb["hash_xor"]) == (bf["count"], bf["hash_sum"], bf["hash_xor"]), (k, e)
        assert al["count"] == bf["maps"], (k, e)


def test_brute_force_six_vertex_patterns():
    g = gg.gnp(8, 0.7, seed=5)
    for name in ["6-cycle", "6-clique"]:
        k, e = P.NAMED[name]
        bf = oracle.brute_force(g.row_ptr, g.col, k, e)
        sb = oracle.enumerate_query(g.row_ptr, g.col, k, e)
        assert (sb["count"], sb["hash_sum"], sb["hash_xor"]) == (bf["count"], bf["hash_sum"], bf["hash_xor"])
    for pat in P.random_patterns(3, seed=9, kmin=6, kmax=6):
        bf = oracle.brute_force(g.row_ptr, g.col, pat["k"], pat["edges"])
        sb = oracle.enumerate_query(g.row_ptr, g.col, pat["k"], pat["edges"])
        assert (sb["count"], sb["hash_sum"], sb["hash_xor"]) == (bf["count"], bf["hash_sum"], bf["hash_xor"])


@pytest.fixture(scope="module")
def chung_lu_16k():
    return gg.chung_lu(16384, 16, 2.5, seed=1, exact=True)


def test_trace_identities_chung_lu(chung_lu_16k):
    g = chung_lu_16k
    assert oracle.enumerate_query(g.row_ptr, g.col, *P.NAMED["triangle"])["count"] == cf.triangles(g)
    assert oracle.enumerate_query(g.row_ptr, g.col, *P.NAMED["4-cycle"])["count"] == cf.four_cycles(g)
    assert oracle.enumerate_query(g.row_ptr, g.col, *P.NAMED["diamond"])["count"] == cf.diamonds(g)


def test_trace_identities_rmat():
    g = gg.rmat(11, 8, seed=3)
    for name, fn in [("triangle", cf.triangles), ("4-cycle", cf.four_cycles), ("diamond", cf.diamonds)]:
        assert oracle.enumerate_query(g.row_ptr, g.col, *P.NAMED[name])["count"] == fn(g), name


def test_root_slices_partition():
    g = gg.chung_lu(4096, 12, 2.5, seed=7)
    for name in ["triangle", "4-cycle", "house"]:
        k, e = P.NAMED[name]
        full = oracle.enumerate_query(g.row_ptr, g.col, k, e)
        S = 8
        cs, hs, hx = 0, 0, 0
        for s in range(S):
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, slice_count=S, slice_id=s)
            cs += r["count"]
            hs = (hs + r["hash_sum"]) & M64
            hx ^= r["hash_xor"]
        assert (cs, hs, hx) == (full["count"], full["hash_sum"], full["hash_xor"]), name


def test_results_independent_of_order():
    g = gg.gnp(30, 0.35, seed=4)
    k, e = P.NAMED["house"]
    ref = oracle.enumerate_query(g.row_ptr, g.col, k, e)
    adj = {frozenset(x) for x in e}
    n_orders = 0
    for order in itertools.permutations(range(k)):
        if any(not any(frozenset((order[p], order[i])) in adj for p in range(i)) for i in range(1, k)):
            with pytest.raises(ValueError):
                oracle.enumerate_query(g.row_ptr, g.col, k, e, order=order)
            continue
        r = oracle.enumerate_query(g.row_ptr, g.col, k, e, order=order)
        assert (r["count"], r["hash_sum"], r["hash_xor"]) == (ref["count"], ref["hash_sum"], ref["hash_xor"])
        n_orders += 1
    assert n_orders > 10


def _brute_level_counts(g, k, e, order, pairs):
    """Partial maps of each prefix of ``order``: injective, keeping the induced
    prefix edges, and satisfying constraints with both ends in the prefix."""
    n = g.n
    rank = oracle.ranks(g.row_ptr)
    adj = set()
    for u in range(n):
        for x in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            adj.add((u, int(g.col[x])))
    out = []
    for d in range(1, k + 1):
        pre = list(order[:d])
        pe = [(a, b) for a, b in e if a in pre and b in pre]
        pp = [(a, b) for a, b in pairs if a in pre and b in pre]
        c = 0
        for img in itertools.permutations(range(n), d):
            f = dict(zip(pre, img))
            if all((f[a], f[b]) in adj for a, b in pe) and all(rank[f[a]] < rank[f[b]] for a, b in pp):
                c += 1
        out.append(c)
    return out


def test_level_counts_match_brute_force():
    g = gg.gnp(9, 0.5, seed=8)
    for name, order in [("house", (4, 0, 1, 2, 3)), ("diamond", (1, 2, 0, 3)), ("4-cycle", (0, 1, 2, 3))]:
        k, e = P.NAMED[name]
        pairs = oracle.sb_pairs(k, e)
        r = oracle.enumerate_query(g.row_ptr, g.col, k, e, order=order)
        assert r["level_counts"][:k] == _brute_level_counts(g, k, e, order, pairs), name


def test_explicit_sb_pairs_give_same_result():
    """Any valid constraint set gives the same subgraphs: here the constraints
    of an isomorphic relabelling of the 4-cycle, mapped back."""
    g = gg.gnp(25, 0.4, seed=6)
    k, e = P.NAMED["4-cycle"]
    ref = oracle.enumerate_query(g.row_ptr, g.col, k, e)
    # rotate the query labels by one: constraints of the rotated query, mapped back
    rot = [(a + 1) % 4 for a in range(4)]
    inv = {rot[a]: a for a in range(4)}
    re_ = [(rot[a], rot[b]) for a, b in e]
    pairs = [(inv[a], inv[b]) for a, b in oracle.sb_pairs(k, re_)]
    alt = oracle.enumerate_query(g.row_ptr, g.col, k, e, sb_pairs=pairs)
    assert (alt["count"], alt["hash_sum"], alt["hash_xor"]) == (ref["count"], ref["hash_sum"], ref["hash_xor"])
    # no constraints: every map
    none = oracle.enumerate_query(g.row_ptr, g.col, k, e, sb_pairs=[])
    assert none["count"] == 8 * ref["count"]


def test_csr_hygiene_checks():
    g = gg.gnp(12, 0.5, seed=3)
    assert oracle.check_csr(g.row_ptr, g.col) == 0
    rp, col = g.row_ptr.copy(), g.col.copy()
    u = int(np.argmax(np.diff(rp)))
    a, b = int(rp[u]), int(rp[u + 1])
    c = col.copy()
    c[a], c[a + 1] = c[a + 1], c[a]
    assert oracle.check_csr(rp, c) == 1
    c = col.copy()
    c[a + 1] = c[a]
    assert oracle.check_csr(rp, c) in (1, 4)
    c = col.copy()
    c[a] = u if u < c[a + 1] else c[a]
    if c[a] == u:
        assert oracle.check_csr(rp, c) in (2, 4)
    c = col.copy()
    c[b - 1] = 12
    assert oracle.check_csr(rp, c) == 3
    # drop one direction of an edge: asymmetric
    e = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    rp2 = e.row_ptr.copy()
    col2 = e.col.copy()
    col2[0] = 2  # row 0 says 0-2, row 2 has no 0
    assert oracle.check_csr(rp2, col2) == 4


def test_mix_is_a_bijection_on_samples():
    xs = [0, 1, 2, 3, 1 << 32, (1 << 64) - 1, 0x123456789ABCDEF0]
    ys = [oracle.mix64(x) for x in xs]
    assert len(set(ys)) == len(xs)


def test_slices_of_any_query_vertex_partition():
    g = gg.chung_lu(2048, 10, 2.5, seed=12)
    k, e = P.NAMED["house"]
    full = oracle.enumerate_query(g.row_ptr, g.col, k, e)
    for sv in range(k):
        cs, hs, hx = 0, 0, 0
        for s in range(5):
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, slice_count=5, slice_id=s, slice_vertex=sv)
            cs += r["count"]
            hs = (hs + r["hash_sum"]) & M64
            hx ^= r["hash_xor"]
        assert (cs, hs, hx) == (full["count"], full["hash_sum"], full["hash_xor"]), sv


def test_pair_slices_partition_and_match_direct_filter():
    """Slices on an ordered pair of query vertices partition the matches, and on a
    tiny graph each slice holds exactly the SB-satisfying maps whose pair of image
    ranks hashes into it (maps enumerated directly with itertools)."""
    import itertools

    g = gg.chung_lu(2048, 10, 2.5, seed=12)
    k, e = P.NAMED["house"]
    full = oracle.enumerate_query(g.row_ptr, g.col, k, e)
    for pair in [(0, 1), (4, 2), (3, 0)]:
        cs, hs, hx = 0, 0, 0
        for s in range(6):
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, slice_count=6, slice_id=s, slice_pair=pair)
            cs += r["count"]
            hs = (hs + r["hash_sum"]) & M64
            hx ^= r["hash_xor"]
        assert (cs, hs, hx) == (full["count"], full["hash_sum"], full["hash_xor"]), pair

    t = gg.gnp(9, 0.55, seed=3)
    rank = oracle.ranks(t.row_ptr)
    adj = {(u, int(v)) for u in range(t.n) for v in t.col[t.row_ptr[u]:t.row_ptr[u + 1]]}
    k, e = P.NAMED["diamond"]
    sb = oracle.sb_pairs(k, e)
    maps = [f for f in itertools.permutations(range(t.n), k)
            if all((f[a], f[b]) in adj for a, b in e) and all(rank[f[a]] < rank[f[b]] for a, b in sb)]
    for pair in [(0, 3), (2, 1)]:
        for s in range(3):
            want = sum(1 for f in maps
                       if oracle.mix64((int(rank[f[pair[0]]]) << 32) | int(rank[f[pair[1]]])) % 3 == s)
            got = oracle.enumerate_query(t.row_ptr, t.col, k, e, slice_count=3, slice_id=s, slice_pair=pair)
            assert got["count"] == want, (pair, s)


def test_strided_and_double_slices_partition_and_match_direct_filter():
    """Strided vertex slices (rank mod S) partition the matches for any query
    vertex; a second vertex slice on another query vertex splits each slice again,
    so the S1 * S2 double slices also partition them, and the double slice
    (a in s1 of S1, b in s2 of S2) is the same set whichever vertex takes the
    first role.  On a tiny graph every slice holds exactly the SB-satisfying maps
    picked out by the rank condition (maps enumerated with itertools)."""
    import itertools

    g = gg.chung_lu(2048, 10, 2.5, seed=12)
    k, e = P.NAMED["house"]
    full = oracle.enumerate_query(g.row_ptr, g.col, k, e)
    want = (full["count"], full["hash_sum"], full["hash_xor"])
    for sv in (0, 2, 4):
        acc = [0, 0, 0]
        for s in range(7):
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, slice_count=7, slice_id=s, slice_vertex=sv,
                                       slice_mode=1)
            acc = [acc[0] + r["count"], (acc[1] + r["hash_sum"]) & M64, acc[2] ^ r["hash_xor"]]
        assert tuple(acc) == want, sv
    acc = [0, 0, 0]
    for s1 in range(3):
        for s2 in range(4):
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, slice_count=3, slice_id=s1, slice_vertex=1,
                                       slice_mode=1, slice2=(3, 4, s2))
            swapped = oracle.enumerate_query(g.row_ptr, g.col, k, e, slice_count=4, slice_id=s2, slice_vertex=3,
                                             slice_mode=1, slice2=(1, 3, s1))
            assert (r["count"], r["hash_sum"], r["hash_xor"]) == \
                (swapped["count"], swapped["hash_sum"], swapped["hash_xor"]), (s1, s2)
            acc = [acc[0] + r["count"], (acc[1] + r["hash_sum"]) & M64, acc[2] ^ r["hash_xor"]]
    assert tuple(acc) == want

    t = gg.gnp(9, 0.55, seed=3)
    rank = oracle.ranks(t.row_ptr)
    adj = {(u, int(v)) for u in range(t.n) for v in t.col[t.row_ptr[u]:t.row_ptr[u + 1]]}
    k, e = P.NAMED["diamond"]
    sb = oracle.sb_pairs(k, e)
    maps = [f for f in itertools.permutations(range(t.n), k)
            if all((f[a], f[b]) in adj for a, b in e) and all(rank[f[a]] < rank[f[b]] for a, b in sb)]
    for a, b in [(0, 3), (2, 1)]:
        for s1 in range(2):
            for s2 in range(3):
                want_n = sum(1 for f in maps if rank[f[a]] % 2 == s1 and rank[f[b]] % 3 == s2)
                got = oracle.enumerate_query(t.row_ptr, t.col, k, e, slice_count=2, slice_id=s1, slice_vertex=a,
                                             slice_mode=1, slice2=(b, 3, s2))
                assert got["count"] == want_n, (a, b, s1, s2)


def test_given_ranks_give_the_same_result():
    g = gg.chung_lu(3000, 8, 2.4, seed=17)
    k, e = P.NAMED["diamond"]
    rk = oracle.ranks(g.row_ptr)
    for kw in [{}, dict(slice_count=5, slice_id=2, slice_mode=1), dict(slice_count=4, slice_id=1, slice_vertex=2)]:
        assert oracle.enumerate_query(g.row_ptr, g.col, k, e, ranks=rk, **kw) == \
            oracle.enumerate_query(g.row_ptr, g.col, k, e, **kw)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_induced_mode_and_motif_brute_force(k):
    """The oracle's induced mode counts, per pattern, the vertex sets whose induced
    subgraph is isomorphic to it: equal to the brute-force motif census (every
    k-subset of a tiny graph), whose non-induced column equals the plain oracle;
    every connected k-subset is counted exactly once over the classes."""
    import itertools

    for seed, n, p in [(1, 10, 0.5), (2, 11, 0.35)]:
        g = gg.gnp(n, p, seed=seed)
        census = oracle.motif_counts(g.row_ptr, g.col, k)
        adj = {(u, int(v)) for u in range(n) for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]}
        conn = 0
        for X in itertools.combinations(range(n), k):
            ind = [(a, b) for a in range(k) for b in range(a + 1, k) if (X[a], X[b]) in adj]
            conn += oracle._connected(k, ind)
        assert sum(v[1] for v in census.values()) == conn
        for key, (nonind, induced) in census.items():
            e = list(key)
            assert oracle.enumerate_query(g.row_ptr, g.col, k, e)["count"] == nonind, key
            assert oracle.enumerate_query(g.row_ptr, g.col, k, e, induced=True)["count"] == induced, key
    K = gg.complete(7)
    clique = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    assert oracle.enumerate_query(K.row_ptr, K.col, 4, clique, induced=True)["count"] == 35
    assert oracle.enumerate_query(K.row_ptr, K.col, 4, [(0, 1), (1, 2), (2, 3)], induced=True)["count"] == 0


def test_labelled_matching_brute_force_and_closed_forms():
    """Labelled queries: every query vertex's image carries its label (-1: any).
    A match is an injective edge- and label-preserving map, counted once per class
    under the automorphisms of q that keep its labels (-1 counting as a label of
    its own).  Brute force over all injective maps of tiny labelled graphs divided
    by that group's order; uniform labels equal the unlabelled count; and in K_n
    with a vertices labelled 0 and b labelled 1 the triangles labelled (0, 0, 1)
    number C(a, 2) * b."""
    import itertools
    import math

    for seed, n, p in [(1, 9, 0.5), (2, 10, 0.4)]:
        g = gg.gnp(n, p, seed=seed)
        lab = [(u * 7 + seed) % 3 for u in range(n)]
        adj = {(u, int(v)) for u in range(n) for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]}
        for name, ql in [("triangle", [0, 1, 1]), ("4-cycle", [0, 1, 0, 1]), ("diamond", [2, 0, 0, -1]),
                         ("4-path", [1, -1, -1, 2])]:
            k, e = P.NAMED[name]
            qadj = {(a, b) for a, b in e} | {(b, a) for a, b in e}
            aut = sum(1 for s_ in itertools.permutations(range(k))
                      if all((s_[a], s_[b]) in qadj for a, b in e) and all(ql[s_[i]] == ql[i] for i in range(k)))
            maps = sum(1 for f in itertools.permutations(range(n), k)
                       if all((f[a], f[b]) in adj for a, b in e) and
                       all(q < 0 or lab[f[i]] == q for i, q in enumerate(ql)))
            assert maps % aut == 0
            got = oracle.enumerate_query(g.row_ptr, g.col, k, e, vlabels=lab, qlabels=ql)
            assert got["count"] == maps // aut, (seed, name)
            same = oracle.enumerate_query(g.row_ptr, g.col, k, e, vlabels=[5] * n, qlabels=[5] * k)
            assert same == oracle.enumerate_query(g.row_ptr, g.col, k, e), name
    K = gg.complete(9)
    lab = [0] * 4 + [1] * 5
    k, e = P.NAMED["triangle"]
    assert oracle.enumerate_query(K.row_ptr, K.col, k, e, vlabels=lab, qlabels=[0, 0, 1])["count"] == \
        math.comb(4, 2) * 5


def _relabelled_entry_index(g):
    """entry[(x, y)] = position of the pair in the CSR relabelled by degree rank
    (rows in rank order, each list sorted by rank), built directly."""
    rank = oracle.ranks(g.row_ptr)
    order = sorted(range(g.n), key=lambda u: int(rank[u]))
    entry, e = {}, 0
    for u in order:
        for v in sorted((int(x) for x in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]), key=lambda z: int(rank[z])):
            entry[(u, v)] = e
            e += 1
    return rank, entry


def test_strided_pair_slices_partition_and_match_the_relabelled_csr():
    """A strided pair slice keeps the maps whose pair (f(a), f(b)) sits at an entry
    e of the rank-relabelled CSR with e mod S == s: on a tiny graph each slice is
    exactly those SB-satisfying maps (entries computed from an explicitly built
    relabelled CSR); the slices partition the matches, for the order's first
    pair and for a later pair; a second pair slice splits them again."""
    import itertools

    t = gg.gnp(10, 0.5, seed=7)
    rank, entry = _relabelled_entry_index(t)
    adj = {(u, int(v)) for u in range(t.n) for v in t.col[t.row_ptr[u]:t.row_ptr[u + 1]]}
    k, e = P.NAMED["diamond"]
    sb = oracle.sb_pairs(k, e)
    maps = [f for f in itertools.permutations(range(t.n), k)
            if all((f[a], f[b]) in adj for a, b in e) and all(rank[f[a]] < rank[f[b]] for a, b in sb)]
    for order, pair in [([1, 2, 0, 3], (1, 2)), ([0, 1, 2, 3], (2, 3)), ([3, 1, 2, 0], (2, 0))]:
        for s in range(5):
            want = sum(1 for f in maps if entry[(f[pair[0]], f[pair[1]])] % 5 == s)
            got = oracle.enumerate_query(t.row_ptr, t.col, k, e, order=order, slice_count=5, slice_id=s,
                                         slice_pair=pair, slice_mode=1)
            assert got["count"] == want, (order, pair, s)
    g = gg.chung_lu(2000, 9, 2.4, seed=12)
    for name, order in [("house", None), ("4-cycle", [1, 2, 3, 0]), ("tailed-triangle", [2, 3, 0, 1])]:
        k, e = P.NAMED[name]
        full = oracle.enumerate_query(g.row_ptr, g.col, k, e)
        o = order or [0, 1, 2, 3, 4][:k]
        acc = [0, 0, 0]
        for s in range(7):
            r = oracle.enumerate_query(g.row_ptr, g.col, k, e, order=o, slice_count=7, slice_id=s,
                                       slice_pair=(o[0], o[1]), slice_mode=1)
            acc = [acc[0] + r["count"], (acc[1] + r["hash_sum"]) & M64, acc[2] ^ r["hash_xor"]]
        assert tuple(acc) == (full["count"], full["hash_sum"], full["hash_xor"]), name
    # double: first pair of one order and first pair of another, in either role
    k, e = P.NAMED["house"]
    oa, ob = [0, 1, 2, 3, 4], [3, 2, 1, 0, 4]
    full = oracle.enumerate_query(g.row_ptr, g.col, k, e)
    acc = [0, 0, 0]
    for s1 in range(3):
        for s2 in range(2):
            a = oracle.enumerate_query(g.row_ptr, g.col, k, e, order=oa, slice_count=3, slice_id=s1,
                                       slice_pair=(0, 1), slice_mode=1, slice2=(3, 2, 2, s2))
            b = oracle.enumerate_query(g.row_ptr, g.col, k, e, order=ob, slice_count=2, slice_id=s2,
                                       slice_pair=(3, 2), slice_mode=1, slice2=(0, 1, 3, s1))
            assert (a["count"], a["hash_sum"], a["hash_xor"]) == (b["count"], b["hash_sum"], b["hash_xor"])
            acc = [acc[0] + a["count"], (acc[1] + a["hash_sum"]) & M64, acc[2] ^ a["hash_xor"]]
    assert tuple(acc) == (full["count"], full["hash_sum"], full["hash_xor"])


DIRECTED = {
    "cycle3": (3, [(0, 1), (1, 2), (2, 0)]),
    "transitive3": (3, [(0, 1), (1, 2), (0, 2)]),
    "path2": (3, [(0, 1), (1, 2)]),
    "in-star": (4, [(1, 0), (2, 0), (3, 0)]),
    "recip-tail": (3, [(0, 1), (1, 0), (1, 2)]),
    "bifan": (4, [(0, 2), (0, 3), (1, 2), (1, 3)]),
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
}


def _arcs(d):
    return {(u, int(v)) for u in range(d.n) for v in d.out_col[d.out_rp[u]:d.out_rp[u + 1]]}


def test_directed_matching_brute_force_and_closed_forms():
    """Directed queries on directed graphs: a match is an injective map keeping
    every query edge's direction, counted once per class of the automorphisms
    that keep directions.  Brute force over all injective maps of tiny digraphs
    divided by that group's order; closed forms on larger ones: directed 3-cycles
    number tr(A^3)/3, transitive triangles sum over arcs a->c of (A^2)_ac, and
    directed 2-paths a->b->c (a != c) sum over b of in(b)*out(b) minus the
    reciprocated pairs at b; with every edge reciprocated, a fully reciprocated
    query counts what the undirected query counts."""
    import itertools

    for seed, n, p, pb in [(1, 8, 0.5, 0.3), (2, 9, 0.45, 0.0), (3, 8, 0.6, 0.6)]:
        d = gg.orient(gg.gnp(n, p, seed=seed), pb, seed=seed + 10)
        arcs = _arcs(d)
        for name, (k, e) in DIRECTED.items():
            aut = sum(1 for s_ in itertools.permutations(range(k))
                      if {(s_[a], s_[b]) for a, b in e} == set(e))
            assert oracle.automorphisms_directed(k, e) == aut, name
            maps = sum(1 for f in itertools.permutations(range(n), k) if all((f[a], f[b]) in arcs for a, b in e))
            assert maps % aut == 0
            got = oracle.enumerate_directed(d.row_ptr, d.col, d.out_rp, d.out_col, k, e)
            assert got["count"] == maps // aut, (seed, name, got["count"], maps // aut)
    import scipy.sparse as sp

    d = gg.orient(gg.chung_lu(2000, 10, 2.4, seed=7), 0.25, seed=8)
    A = sp.csr_matrix((np.ones(d.arcs, dtype=np.int64), d.out_col, d.out_rp), shape=(d.n, d.n))
    A2 = A @ A
    run = lambda name: oracle.enumerate_directed(d.row_ptr, d.col, d.out_rp, d.out_col, *DIRECTED[name])["count"]
    assert run("cycle3") == int((A2 @ A).diagonal().sum()) // 3
    assert run("transitive3") == int(A.multiply(A2).sum())
    recip = int(A.multiply(A.T).sum())
    indeg, outdeg = np.asarray(A.sum(axis=0)).ravel(), np.asarray(A.sum(axis=1)).ravel()
    assert run("path2") == int((indeg * outdeg).sum()) - recip
    u = gg.chung_lu(600, 8, 2.4, seed=9)
    full = gg.orient(u, 1.0, seed=1)
    for name in ["triangle", "4-cycle", "diamond"]:
        k, e = P.NAMED[name]
        both = [x for a, b in e for x in ((a, b), (b, a))]
        assert oracle.enumerate_directed(full.row_ptr, full.col, full.out_rp, full.out_col, k, both) == \
            oracle.enumerate_query(u.row_ptr, u.col, k, e), name


def _dfs_paths(g, s, t, L):
    """Simple s-t paths of exactly L edges, by depth-first search."""
    adj = [list(map(int, g.col[g.row_ptr[u]:g.row_ptr[u + 1]])) for u in range(g.n)]
    cnt = 0
    stack = [(s, (s,))]
    while stack:
        u, path = stack.pop()
        if len(path) == L + 1:
            cnt += u == t
            continue
        for v in adj[u]:
            if v not in path and (v != t or len(path) == L):
                stack.append((v, path + (v,)))
    return cnt


def pinned_path_counts(g, s, t, max_hops, ranks=None):
    """The oracle's count of the path query 0 - ... - L, every map (no symmetry
    breaking), vertex 0 pinned to s and vertex L to t by strided slices of
    count n (one rank each): the hop-constrained path counts."""
    rk = oracle.ranks(g.row_ptr) if ranks is None else ranks
    out = [0]
    for L in range(1, max_hops + 1):
        e = [(i, i + 1) for i in range(L)]
        r = oracle.enumerate_query(g.row_ptr, g.col, L + 1, e, mode=oracle.MODE_ALL, order=list(range(L + 1)),
                                   slice_count=g.n, slice_id=int(rk[s]), slice_vertex=0, slice_mode=1,
                                   slice2=(L, g.n, int(rk[t])), ranks=rk)
        out.append(r["count"])
    return out


def test_pinned_path_counts():
    """Hop-constrained s-t paths: the pinned all-maps path queries equal a
    depth-first search on random graphs, and on K_n the paths of L edges number
    (n-2)! / (n-1-L)! (the ordered choice of the L-1 inner vertices)."""
    import math

    for seed, n, p in [(1, 12, 0.35), (2, 14, 0.3)]:
        g = gg.gnp(n, p, seed=seed)
        for s, t in [(0, 1), (3, 7)]:
            got = pinned_path_counts(g, s, t, 5)
            assert got == [0] + [_dfs_paths(g, s, t, L) for L in range(1, 6)], (seed, s, t)
    K = gg.complete(8)
    assert pinned_path_counts(K, 2, 5, 7) == [0] + [math.factorial(6) // math.factorial(7 - L) for L in range(1, 8)]
