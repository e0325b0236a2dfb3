"""Algorithm 1 (OptimalExecutionPlan, Section 3.3) on the host: bushy plans over
connected edge sets, stars as join units, each join's physical setting from the
settings equation, costs M(l) + M(r) + |R(q')| plus machines * |E_G| for a
pulled join or |R(l)| + |R(r)| for a PUSH-JOIN.  Checked here against an
exhaustive top-down search over every join tree, written independently from
the same definitions, with synthetic degree statistics (no GPU)."""
import functools
import itertools
import math

import pytest

import paper_2103_14294_amd as H
from graphgen import patterns as P

NAMES = ["edge", "wedge", "triangle", "3-star", "4-path", "4-cycle", "tailed-triangle", "diamond", "4-clique",
         "5-cycle", "house", "5-clique", "6-cycle"]

# two degree sequences: a flat one and a skewed one (sum_u d_u^p, p = 0..7)
STATS = {
    "flat": [10 ** 6 * 12.0 ** p for p in range(8)],
    "skewed": [float(sum(c * d ** p for d, c in [(2, 5 * 10 ** 5), (20, 4 * 10 ** 5), (400, 10 ** 5), (20000, 100)]))
               for p in range(8)],
}


def stats(name):
    m = STATS[name]
    return {"n": int(m[0]), "nnz": int(m[1]), "degree_moments": m}


def sb_fraction(verts, sb):
    cons = [(a, b) for a, b in sb if a in verts and b in verts]
    if not cons:
        return 1.0
    vs = sorted(verts)
    good = tot = 0
    for perm in itertools.permutations(range(len(vs))):
        r = dict(zip(vs, perm))
        tot += 1
        good += all(r[a] < r[b] for a, b in cons)
    return good / tot


class Search:
    """Every join tree of a query, top-down, from the definitions."""

    def __init__(self, k, edges, sb, st, machines):
        self.k, self.edges, self.sb, self.machines = k, [tuple(e) for e in edges], sb, machines
        self.M, self.two_m = st["degree_moments"], float(st["nnz"])

    def verts(self, es):
        return {v for e in es for v in e}

    def connected(self, es):
        es = list(es)
        seen = {es[0][0]}
        changed = True
        while changed:
            changed = False
            for a, b in es:
                if (a in seen) != (b in seen):
                    seen |= {a, b}
                    changed = True
        return seen == self.verts(es)

    def est(self, es):
        vs = self.verts(es)
        deg = {v: sum(v in e for e in es) for v in vs}
        logv = sum(math.log(self.M[min(d, 7)]) for d in deg.values()) - len(es) * math.log(self.two_m)
        return math.exp(logv) * sb_fraction(vs, self.sb)

    def star(self, es):
        """(centre candidates) of a star, or [] when es is not a star."""
        if len(es) == 1:
            return list(es[0])
        common = set(es[0])
        for e in es[1:]:
            common &= set(e)
        return sorted(common)

    def kind(self, l, r):
        vl = self.verts(l)
        cs = self.star(r)
        for c in cs:
            leaves = self.verts(r) - {c}
            if c not in vl and leaves <= vl:
                return "extend"
        for c in cs:
            if c in vl:
                return "pull_hash"
        return "push"

    @functools.lru_cache(maxsize=None)
    def cost(self, es):
        es = tuple(sorted(es))
        if self.star(list(es)):
            return self.est(es)
        best = math.inf
        n = len(es)
        for mask in range(1, (1 << n) - 1):
            l = tuple(es[i] for i in range(n) if (mask >> i) & 1)
            r = tuple(es[i] for i in range(n) if not (mask >> i) & 1)
            if not self.connected(l) or not self.connected(r):
                continue
            kind = self.kind(list(l), list(r))
            comm = self.machines * self.two_m / 2 if kind != "push" else self.est(l) + self.est(r)
            best = min(best, self.cost(l) + self.cost(r) + self.est(es) + comm)
        return best


def edges_of(mask, edges):
    return [tuple(edges[i]) for i in range(len(edges)) if (mask >> i) & 1]


@pytest.mark.parametrize("machines", [0.0, 1.0, 1e-3, 1e6])
@pytest.mark.parametrize("sname", ["flat", "skewed"])
@pytest.mark.parametrize("name", NAMES)
def test_dp_matches_exhaustive_search(name, sname, machines):
    k, e = P.NAMED[name]
    st = stats(sname)
    p = H.plan_bushy(None, k, e, machines=machines, stats=st)
    nodes = p.bushy_nodes()
    sb = [tuple(x) for x in p.info()["sb_pairs"]]
    edges = [tuple(sorted(x)) for x in e]
    S = Search(k, edges, sb, st, machines)
    root = nodes[-1]
    assert root["edge_mask"] == (1 << len(e)) - 1
    want = S.cost(tuple(sorted(edges)))
    assert root["cost"] == pytest.approx(want, rel=1e-9), (name, root["cost"], want)
    # the recovered tree: parts partition their parent's edges, are connected,
    # carry their own estimates, costs add up, and the kinds follow the settings
    for i, nd in enumerate(nodes):
        es = edges_of(nd["edge_mask"], edges)
        assert S.connected(es)
        assert nd["est_rows"] == pytest.approx(S.est(tuple(es)), rel=1e-9)
        assert nd["vertex_mask"] == sum(1 << v for v in S.verts(es))
        if nd["kind"] == "unit":
            assert S.star(es) and nd["left"] == nd["right"] == -1
            assert nd["cost"] == pytest.approx(nd["est_rows"], rel=1e-12)
            continue
        assert not S.star(es), "a star is a join unit and never split"
        L, R = nodes[nd["left"]], nodes[nd["right"]]
        assert nd["left"] < i and nd["right"] < i
        assert L["edge_mask"] & R["edge_mask"] == 0 and L["edge_mask"] | R["edge_mask"] == nd["edge_mask"]
        le, re_ = edges_of(L["edge_mask"], edges), edges_of(R["edge_mask"], edges)
        assert nd["kind"] == S.kind(le, re_), (name, i)
        comm = machines * st["nnz"] / 2 if nd["kind"] != "push" else L["est_rows"] + R["est_rows"]
        assert nd["cost"] == pytest.approx(L["cost"] + R["cost"] + nd["est_rows"] + comm, rel=1e-9)
        if nd["kind"] != "push":
            # the star is the right part; its centre is the join's
            c = nd["star_root"]
            assert c in S.star(re_)
            assert (c in S.verts(le)) == (nd["kind"] == "pull_hash")


@pytest.mark.parametrize("name", ["edge", "wedge", "3-star"])
def test_a_star_query_is_one_unit(name):
    k, e = P.NAMED[name]
    nodes = H.plan_bushy(None, k, e, stats=stats("skewed")).bushy_nodes()
    assert len(nodes) == 1 and nodes[0]["kind"] == "unit"


def test_dear_pulls_push_where_they_can():
    """Pulling at a huge price: a path splits into two paths joined by a
    PUSH-JOIN; a triangle has no pushed split (every split has a star side whose
    leaves the other part holds), so it stays pulled."""
    k, e = P.NAMED["4-path"]
    nodes = H.plan_bushy(None, k, e, machines=1e12, stats=stats("flat")).bushy_nodes()
    assert nodes[-1]["kind"] == "push"
    k, e = P.NAMED["triangle"]
    nodes = H.plan_bushy(None, k, e, machines=1e12, stats=stats("flat")).bushy_nodes()
    assert nodes[-1]["kind"] in ("extend", "pull_hash")


def test_bushy_planning_errors():
    k, e = P.NAMED["triangle"]
    with pytest.raises(H.HugeError) as ei:
        H.plan_bushy(None, k, e)  # no graph, no statistics
    assert ei.value.name == "HUGE_EINVAL"
    with pytest.raises(H.HugeError) as ei:
        H.plan_bushy(None, k, e, machines=-1.0, stats=stats("flat"))
    assert ei.value.name == "HUGE_EINVAL"
    k8 = 7
    e8 = [(a, b) for a in range(k8) for b in range(a + 1, k8)][:16]
    with pytest.raises(H.HugeError) as ei:
        H.plan_bushy(None, k8, e8, stats=stats("flat"))
    assert ei.value.name == "HUGE_EQUERY"
    # a plain plan has no join tree
    with pytest.raises(H.HugeError) as ei:
        H.plan(None, k, e).bushy_nodes()
    assert ei.value.name == "HUGE_EINVAL"


# logical plans given by the caller (Remark 3.2): (query edges, joins as edge masks, kinds root-last)
TREES = {
    # two wedges pushed together, then a complete star join closes a 6-cycle
    "extend-over-push": ([(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0)],
                         [(0b000011, 0b001100), (0b001111, 0b110000)], ["push", "extend"]),
    # the same path closed by one verified edge (a 5-cycle)
    "verify-over-push": ([(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)],
                         [(0b00011, 0b01100), (0b01111, 0b10000)], ["push", "pull_hash"]),
    # a star whose centre is in the path: one edge verified, one leaf grown
    "grow-over-push": ([(0, 1), (1, 2), (2, 3), (3, 4), (0, 4), (0, 5)],
                       [(0b000011, 0b001100), (0b001111, 0b110000)], ["push", "pull_hash"]),
    # a PUSH-JOIN of a PUSH-JOIN and a triangle (a wedge closed by a verified edge)
    "push-of-push": ([(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (0, 4)],
                     [(0b0000011, 0b0001100), (0b0110000, 0b1000000), (0b0001111, 0b1110000)],
                     ["push", "pull_hash", "push"]),
}


@pytest.mark.parametrize("name", sorted(TREES))
def test_given_trees_get_their_settings(name):
    e, joins, kinds = TREES[name]
    k = 1 + max(max(x) for x in e)
    st = stats("skewed")
    p = H.plan_bushy(None, k, e, machines=1.0, stats=st, joins=joins)
    nodes = p.bushy_nodes()
    joins_made = [nd for nd in nodes if nd["kind"] != "unit"]
    assert [nd["kind"] for nd in joins_made] == kinds
    sb = [tuple(x) for x in p.info()["sb_pairs"]]
    S = Search(k, [tuple(sorted(x)) for x in e], sb, st, 1.0)
    for nd in joins_made:
        L, R = nodes[nd["left"]], nodes[nd["right"]]
        assert {L["edge_mask"], R["edge_mask"]} in [set(j) for j in joins]
        comm = st["nnz"] / 2 if nd["kind"] != "push" else L["est_rows"] + R["est_rows"]
        assert nd["cost"] == pytest.approx(L["cost"] + R["cost"] + nd["est_rows"] + comm, rel=1e-9)
        assert nd["est_rows"] == pytest.approx(S.est(tuple(edges_of(nd["edge_mask"], e))), rel=1e-9)


def test_given_tree_errors():
    e = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0)]
    st = stats("flat")
    bad = [
        [(0b000011, 0b000110)],                              # overlapping parts
        [(0b000101, 0b111010)],                              # a disconnected part
        [(0b000111, 0b111000)],                              # leaves that are not stars (3-edge paths)
        [(0b000011, 0b001100)],                              # the root is not split
        [(0b000011, 0b001100), (0b001111, 0b110000), (0b000010, 0b000100)],  # a join outside the tree
        [(0b000011, 0b001100), (0b001111, 0b110000), (0b001111, 0b110000)],  # a part split twice
    ]
    for joins in bad:
        with pytest.raises(H.HugeError) as ei:
            H.plan_bushy(None, 6, e, stats=st, joins=joins)
        assert ei.value.name == "HUGE_EORDER", joins
    # a star part may still be split (into smaller stars)
    p = H.plan_bushy(None, 6, e, stats=st, joins=[(0b000011, 0b001100), (0b001111, 0b110000), (0b000001, 0b000010)])
    assert len(p.bushy_nodes()) == 7
    # a star query needs no join
    assert len(H.plan_bushy(None, 4, P.NAMED["3-star"][1], stats=st, joins=[]).bushy_nodes()) == 1
