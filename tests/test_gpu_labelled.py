"""Labelled graphs and queries (huge_load_csr_labelled, huge_plan_create_labelled):
every query vertex's image carries its label (-1: any), matches counted once per
class under the label-keeping automorphisms; against the oracle's labelled mode,
on every strategy and engine, with slices and induced plans, and closed forms."""
import math

import numpy as np
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import cmp_key, need_gpu, oracle_run

pytestmark = pytest.mark.gpu

CASES = [("triangle", [0, 1, 1]), ("triangle", [2, 2, 2]), ("4-cycle", [0, 1, 0, 1]), ("diamond", [2, 0, 0, -1]),
         ("4-path", [1, -1, -1, 2]), ("house", [0, 0, 1, 1, 2]), ("5-clique", [-1, -1, 0, 0, 1]),
         ("tailed-triangle", [1, 1, -1, 0])]


@pytest.fixture(scope="module")
def H():
    return need_gpu()


@pytest.fixture(scope="module")
def graph(H):
    g = gg.chung_lu(3000, 14, 2.3, seed=91)
    lab = (np.arange(g.n) * 2654435761 % 97 % 3).astype(np.int32)
    return g, lab, H.load(g.row_ptr, g.col, labels=lab)


@pytest.mark.parametrize("name,ql", CASES)
def test_labelled_matches_oracle(H, graph, name, ql):
    g, lab, G = graph
    k, e = P.NAMED[name]
    p = H.plan(G, k, e, labels=ql)
    order = p.info()["order"]
    ref = oracle_run(g, k, e, order=order, vlabels=lab, qlabels=ql)
    for strategy in (0, 1, 2, 5, 6):
        r = H.count(G, p, strategy=strategy)
        assert cmp_key(r, k) == cmp_key(ref, k), (name, strategy)
        assert r["level_counts"][:k] == ref["level_counts"][:k], (name, strategy)
    assert cmp_key(H.count(G, p, engine=H.ENGINE_GRAPH), k) == cmp_key(ref, k)
    s = H.count(G, p, slice_count=3, slice_id=2, slice_vertex=-1, slice_mode=H.SLICE_STRIDE)
    refs = oracle_run(g, k, e, order=order, vlabels=lab, qlabels=ql, slice_count=3, slice_id=2,
                      slice_vertex=order[0], slice_mode=1)
    assert cmp_key(s, k) == cmp_key(refs, k)


def test_labelled_batch_induced_and_enumerate(H, graph):
    g, lab, G = graph
    plans = [H.plan(G, P.NAMED[n][0], P.NAMED[n][1], labels=ql) for n, ql in CASES]
    outs = H.count_batch(G, plans, engine=H.ENGINE_GRAPH)
    for (n, ql), pl, r in zip(CASES, plans, outs):
        k, e = P.NAMED[n]
        ref = oracle_run(g, k, e, order=pl.info()["order"], vlabels=lab, qlabels=ql)
        assert cmp_key(r, k) == cmp_key(ref, k), n
    k, e = P.NAMED["4-path"]
    pi = H.plan(G, k, e, labels=[0, -1, -1, 1], induced=True)
    ref = oracle_run(g, k, e, order=pi.info()["order"], vlabels=lab, qlabels=[0, -1, -1, 1], induced=True)
    assert cmp_key(H.count(G, pi), k) == cmp_key(ref, k)
    pe = H.plan(G, *P.NAMED["triangle"], labels=[0, 1, 1])
    d = H.enumerate_matches(G, pe, buf_rows=4096)
    rows = d["rows"]
    assert rows.shape[0] == d["count"] > 0
    assert (lab[rows[:, 0]] == 0).all() and (lab[rows[:, 1]] == 1).all() and (lab[rows[:, 2]] == 1).all()


def test_labelled_closed_forms_and_errors(H):
    K = gg.complete(9)
    lab = np.array([0] * 4 + [1] * 5, np.int32)
    G = H.load(K.row_ptr, K.col, labels=lab)
    k, e = P.NAMED["triangle"]
    assert H.count(G, H.plan(G, k, e, labels=[0, 0, 1]))["count"] == math.comb(4, 2) * 5
    assert H.count(G, H.plan(G, k, e, labels=[1, 1, 1]))["count"] == math.comb(5, 3)
    assert H.count(G, H.plan(G, k, e, labels=[-1, -1, -1]))["count"] == math.comb(9, 3)
    plain = H.load(K.row_ptr, K.col)
    with pytest.raises(H.HugeError):
        H.count(plain, H.plan(plain, k, e, labels=[0, 0, 1]))
    with pytest.raises(H.HugeError):
        H.count(G, H.plan(G, k, e, labels=[0, 0, 1]), engine=H.ENGINE_PERSISTENT)
