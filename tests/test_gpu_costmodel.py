"""The plain cost model (Algorithm 1 restricted to left-deep worst-case-optimal
plans, with the Chung-Lu estimator) pinned to its definition, recomputed here
independently: per prefix, the product of degree moments over (2m)^edges times
the exact fraction of the prefix's orderings that satisfy its symmetry-breaking
constraints; over the whole query that fraction is 1/|Aut(q)| (the
Grochow-Kellis constraints keep one labelling per automorphism class); the
chosen order minimises the summed estimate, ties to the lexicographically
smallest; and planning is deterministic."""
import itertools
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
from graphgen import patterns as P
from tests.gpu_common import need_gpu

pytestmark = pytest.mark.gpu

NAMES = ["edge", "wedge", "triangle", "4-path", "3-star", "4-cycle", "tailed-triangle", "diamond", "4-clique",
         "5-cycle", "house", "5-clique", "6-cycle"]


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def graph(H):
    g = gg.chung_lu(5000, 12, 2.3, seed=51)
    return g, H.load(g.row_ptr, g.col)


def moments(g):
    d = np.diff(g.row_ptr).astype(np.float64)
    return [float((d ** p).sum()) for p in range(8)]


def sb_fraction(verts, sb):
    """Fraction of the orderings of `verts` that satisfy every constraint a < b
    with both ends in verts (brute force over permutations)."""
    cons = [(a, b) for a, b in sb if a in verts and b in verts]
    if not cons:
        return 1.0
    good = tot = 0
    for perm in itertools.permutations(range(len(verts))):
        rank = {v: perm[i] for i, v in enumerate(verts)}
        tot += 1
        good += all(rank[a] < rank[b] for a, b in cons)
    return good / tot


def estimate(M, nnz, edges, sb, verts):
    deg = {v: sum(1 for a, b in edges if (a == v and b in verts) or (b == v and a in verts)) for v in verts}
    ne = sum(1 for a, b in edges if a in verts and b in verts)
    logv = sum(math.log(M[min(deg[v], 7)]) for v in verts) - ne * math.log(nnz)
    return math.exp(logv) * sb_fraction(verts, sb)


def connected_orders(k, edges):
    adj = {(a, b) for a, b in edges} | {(b, a) for a, b in edges}
    return [list(o) for o in itertools.permutations(range(k))
            if all(any((o[i], o[j]) in adj for j in range(i)) for i in range(1, k))]


@pytest.mark.parametrize("name", NAMES)
def test_estimates_follow_the_definition(H, graph, name):
    g, G = graph
    k, e = P.NAMED[name]
    M = moments(g)
    p = H.plan(G, k, e)
    order = p.info()["order"]
    sb = [tuple(x) for x in p.info()["sb_pairs"]]
    assert sorted(sb) == sorted(tuple(x) for x in oracle.sb_pairs(k, e))
    est = p.estimates()
    for s in range(1, k + 1):
        want = estimate(M, g.nnz, e, sb, order[:s])
        assert est[s - 1] == pytest.approx(want, rel=1e-9), (name, s)
    # the first edge: 2m ordered pairs, halved by a constraint between its ends
    halved = any({a, b} == set(order[:2]) for a, b in sb)
    assert est[1] == pytest.approx(g.nnz / (2 if halved else 1), rel=1e-12)
    # the whole query: the constraints keep exactly 1/|Aut(q)| of the orderings
    naut = len(oracle.automorphisms(k, e))
    plain = estimate(M, g.nnz, e, [], list(range(k)))
    assert est[k - 1] * naut == pytest.approx(plain, rel=1e-9), (name, naut)
    assert sb_fraction(list(range(k)), sb) == pytest.approx(1.0 / naut, rel=1e-12)
    assert p.info()["est_cost"] == pytest.approx(sum(est[1:]), rel=1e-12)


@pytest.mark.parametrize("name", ["4-path", "tailed-triangle", "diamond", "house", "5-cycle"])
def test_chosen_order_minimises_the_estimate(H, graph, name):
    g, G = graph
    k, e = P.NAMED[name]
    M = moments(g)
    sb = [tuple(x) for x in oracle.sb_pairs(k, e)]
    best, best_cost = None, math.inf
    for o in connected_orders(k, e):  # lexicographic
        c = sum(estimate(M, g.nnz, e, sb, o[:s]) for s in range(2, k + 1))
        if c < best_cost * (1 - 1e-12):
            best, best_cost = o, c
    p = H.plan(G, k, e)
    assert p.info()["order"] == best, (name, p.info()["order"], best)
    assert p.info()["est_cost"] == pytest.approx(best_cost, rel=1e-9)


def test_planning_is_deterministic(H, graph):
    _, G = graph
    for name in ["house", "diamond", "6-cycle"]:
        k, e = P.NAMED[name]
        infos = [H.plan(G, k, e).info() for _ in range(3)]
        ests = [H.plan(G, k, e).estimates() for _ in range(3)]
        assert all(i == infos[0] for i in infos), name
        assert all(x == ests[0] for x in ests), name
