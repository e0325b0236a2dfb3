"""Bushy plans on the GPU (Algorithm 1's join trees, Section 3.3; PUSH-JOIN,
Section 4.3; the verify-only EXTEND of pulled hash joins, Section 5.1).

A plan's matches do not depend on its shape, so every tree must give the
oracle's count and set-hashes for the whole query; and every part a tree
materialises (the children of a PUSH-JOIN, and every step above one) must hold
exactly the oracle's matches of that part: its edges, the symmetry-breaking
constraints inside it, injective.  Algorithm 1's `machines` (the k of k |E_G|)
sweeps the trees from all-pulled (0) to as-pushed-as-possible (huge), with
mixed trees in between; a coverage test checks that the sweep runs chains
with verified edges and PUSH-JOINs of units and of chains, and trees given by
the caller run pulled joins over a PUSH-JOIN's table and PUSH-JOINs of
PUSH-JOINs."""
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu

NAMES = ["triangle", "4-path", "4-cycle", "tailed-triangle", "diamond", "4-clique", "5-cycle", "house", "6-cycle",
         "3-star"]
MACHINES = [0.0, 1e-6, 1e-4, 1e-2, 1.0, 1e9]


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def graphs(H):
    out = {}
    for name, g in [("cl", gg.chung_lu(500, 6, 2.5, seed=61)), ("rmat", gg.rmat(8, 5, seed=62))]:
        out[name] = (g, H.load(g.row_ptr, g.col))
    return out


def sub_oracle(g, e, mask, sb):
    """The oracle's matches of the part made of the query edges in `mask`, with
    the symmetry-breaking constraints inside it."""
    es = [tuple(e[i]) for i in range(len(e)) if (mask >> i) & 1]
    vs = sorted({v for x in es for v in x})
    ix = {v: i for i, v in enumerate(vs)}
    sub_e = [(ix[a], ix[b]) for a, b in es]
    sub_sb = [(ix[a], ix[b]) for a, b in sb if a in ix and b in ix]
    return oracle_run(g, len(vs), sub_e, sb_pairs=sub_sb)["count"]


def shapes(nodes):
    """Operator shapes a tree exercises."""
    out = set()
    for nd in nodes:
        if nd["kind"] == "push":
            kinds = {nodes[nd["left"]]["kind"], nodes[nd["right"]]["kind"]}
            out.add("push")
            if "push" in kinds:
                out.add("push-of-push")
            if kinds & {"extend", "pull_hash"}:
                out.add("push-of-chain")
        elif nd["kind"] in ("extend", "pull_hash"):
            below = nodes[nd["left"]]["kind"]
            out.add(nd["kind"])
            if below == "push":
                out.add("pull-over-push")
    return out


def run_case(H, g, G, name, k, e, machines, check_parts=True, joins=None):
    p = H.plan_bushy(G, k, e, machines=machines, joins=joins)
    nodes = p.bushy_nodes()
    r, rows = H.count_bushy(G, p)
    ref = oracle_run(g, k, e)
    assert cmp_key(r, k) == cmp_key(ref, k), (name, machines, [n["kind"] for n in nodes], r["count"], ref["count"])
    assert rows[len(nodes) - 1] == ref["count"]
    # the plain entry point runs the same tree
    assert cmp_key(H.count(G, p), k) == cmp_key(ref, k)
    if check_parts:
        sb = [tuple(x) for x in p.info()["sb_pairs"]]
        for i, nd in enumerate(nodes[:-1]):
            if rows[i] >= 0:
                assert rows[i] == sub_oracle(g, e, nd["edge_mask"], sb), (name, machines, i, nd)
    return nodes


@pytest.mark.parametrize("machines", MACHINES)
@pytest.mark.parametrize("name", NAMES)
def test_bushy_plans_match_oracle(H, graphs, name, machines):
    k, e = P.NAMED[name]
    for gname, (g, G) in graphs.items():
        print("bushy %s machines=%g graph=%s" % (name, machines, gname), flush=True)
        run_case(H, g, G, name, k, e, machines)


def test_bushy_random_patterns_and_coverage(H, graphs):
    """Random 4-6-vertex patterns over the machines sweep: oracle parity, and
    together every operator shape the executor has."""
    g, G = graphs["rmat"]
    seen = set()
    pats = P.random_patterns(14, seed=63, kmin=4, kmax=6)
    for i, pat in enumerate(pats):
        for machines in MACHINES:
            print("bushy random %d k=%d machines=%g" % (i, pat["k"], machines), flush=True)
            nodes = run_case(H, g, G, "random-%d" % i, pat["k"], pat["edges"], machines, check_parts=i < 6)
            seen |= shapes(nodes)
    for k, e in (P.NAMED[n] for n in NAMES):
        for machines in MACHINES:
            seen |= shapes(H.plan_bushy(G, k, e, machines=machines).bushy_nodes())
    want = {"extend", "pull_hash", "push", "push-of-chain"}
    assert want <= seen, want - seen


@pytest.mark.parametrize("tree", ["extend-over-push", "verify-over-push", "grow-over-push", "push-of-push"])
def test_bushy_given_trees(H, graphs, tree):
    """Logical plans given by the caller (Remark 3.2) reach the shapes the
    optimiser's choices above do not: pulled joins over a PUSH-JOIN's table
    (a complete star join, a verify-only EXTEND, a verify plus a grown leaf)
    and a PUSH-JOIN of a PUSH-JOIN with a pulled chain."""
    from tests.test_bushy_plan import TREES

    e, joins, kinds = TREES[tree]
    k = 1 + max(max(x) for x in e)
    for gname, (g, G) in graphs.items():
        print("bushy tree %s graph=%s" % (tree, gname), flush=True)
        nodes = run_case(H, g, G, tree, k, e, 1.0, joins=joins)
        assert [nd["kind"] for nd in nodes if nd["kind"] != "unit"] == kinds
        sh = shapes(nodes)
        assert ("pull-over-push" in sh) == tree.endswith("over-push")
        assert ("push-of-push" in sh) == (tree == "push-of-push")


@pytest.mark.parametrize("name", ["4-path", "house", "6-cycle"])
def test_bushy_vertex_slices_partition(H, graphs, name):
    """A vertex slice filters the sliced vertex wherever it is placed (in every
    part holding it): slices match the oracle's and add up to the whole."""
    g, G = graphs["cl"]
    k, e = P.NAMED[name]
    for machines in (0.0, 1e9):
        p = H.plan_bushy(G, k, e, machines=machines)
        tot = [0, 0, 0]
        for mode in (H.SLICE_MIX, H.SLICE_STRIDE):
            tot = [0, 0, 0]
            for s in range(3):
                r = H.count(G, p, slice_count=3, slice_id=s, slice_vertex=1, slice_mode=mode)
                ref = oracle_run(g, k, e, slice_count=3, slice_id=s, slice_vertex=1, slice_mode=int(mode))
                assert cmp_key(r, k) == cmp_key(ref, k), (name, machines, mode, s)
                tot = [tot[0] + r["count"], (tot[1] + r["hash_sum"]) % (1 << 64), tot[2] ^ r["hash_xor"]]
            assert tuple(tot) == cmp_key(oracle_run(g, k, e), k)


def test_bushy_labelled(H):
    g = gg.chung_lu(1200, 8, 2.4, seed=64)
    import numpy as np

    labels = (np.arange(g.n) * 7 % 3).astype(np.int32)
    G = H.load(g.row_ptr, g.col, labels=labels)
    for name, ql in [("4-path", [0, 1, -1, 1]), ("house", [0, -1, 1, 2, -1])]:
        k, e = P.NAMED[name]
        for machines in (0.0, 1e9):
            p = H.plan_bushy(G, k, e, machines=machines, labels=ql)
            r = H.count(G, p)
            ref = oracle_run(g, k, e, vlabels=labels, qlabels=np.asarray(ql, dtype=np.int32))
            assert cmp_key(r, k) == cmp_key(ref, k), (name, machines)


def test_bushy_errors(H, graphs):
    g, G = graphs["cl"]
    k, e = P.NAMED["house"]
    p = H.plan_bushy(G, k, e, machines=1e9)
    bad = [dict(engine=H.ENGINE_GRAPH), dict(engine=H.ENGINE_PERSISTENT), dict(work_limit=100),
           dict(slice_count=4, slice_vertex=-2), dict(slice_count=4, slice_vertex=-1),
           dict(slice_count=4, slice_vertex=0, slice2=(1, 3, 0)), dict(profile=True)]
    for kw in bad:
        with pytest.raises(H.HugeError) as ei:
            H.count(G, p, **kw)
        assert ei.value.name == "HUGE_EINVAL", kw
    with pytest.raises(H.HugeError):
        H.enumerate_matches(G, p, buf_rows=64)
    with pytest.raises(H.HugeError):
        H.count_batch(G, [p])
