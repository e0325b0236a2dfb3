"""What the trained networks gain over the method without them.

* Cardinality: on the graphs it was trained on (two of the training graphs,
  the networks' intended use: a graph that is queried again and again) and
  for patterns held out of training, the cardinality network estimates
  |R(prefix)| -- the quantity the plain cost model ranks orders by -- with a
  smaller q-error than the Chung-Lu estimate that cost model uses.  True
  sizes are counts of prefix plans on root slices scaled by the slice count,
  as in the training labels.  (On graphs of other
  sizes than those it was trained on the network does not carry over; that
  is measured and reported, not tested.)
* Planning: plans chosen by the work network (with measured verification)
  count exactly the same matches as the cost model's plans and the oracle.
"""
import math
import os
import random
import time

import numpy as np
import pytest

import graphgen as gg
from graphgen import patterns as P
from tests.gpu_common import assert_parity, need_gpu

pytestmark = pytest.mark.gpu

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2103_14294_amd")


@pytest.fixture(scope="module")
def H():
    return need_gpu()


def _qerr(est, true):
    a, b = np.maximum(1.0, est), np.maximum(1.0, true)
    return np.maximum(a / b, b / a)


def test_count_model_beats_chung_lu_on_held_out_patterns(H):
    from paper_2103_14294_amd import learn

    m = H.Model.load(os.path.join(PKG, "mlp_count.npz"))
    seen = {(p["k"], tuple(p["edges"])) for p in P.random_patterns(2100, seed=1, kmin=4, kmax=6, distinct="labelled")}
    pats = [p for p in P.random_patterns(400, seed=4242, kmin=4, kmax=6, distinct="labelled")
            if (p["k"], tuple(p["edges"])) not in seen][:30]
    specs = dict(learn.TRAIN_GRAPHS)
    rng = random.Random(7)
    ws = H.Workspace()
    X, T = [], []
    for g in [learn.make_graph(specs["rmat18"]), learn.make_graph(specs["cl500k"])]:
        G = H.load(g.row_ptr, g.col)
        deadline = time.time() + 40
        for q in pats:
            if time.time() > deadline:
                break
            p = H.plan(G, q["k"], q["edges"])
            prev = float(g.n)
            for s in range(2, q["k"] + 1):
                got = learn.measure_prefix(G, H.plan_prefix(p, s), s, prev, 2.0 * g.m / g.n, 5e8, rng, ws, g.n)
                if got is None:
                    break  # deeper prefixes cost more
                X.append(H.plan_features(G, p, s))
                T.append(got[0])
                prev = max(got[0], 1.0)
        G.free()
    X = np.asarray(X, np.float32)
    T = np.asarray(T)
    assert len(T) >= 40, len(T)
    est_mlp = np.expm1(m.forward(X).astype(np.float64))
    est_cl = np.expm1(X[:, 126].astype(np.float64))  # the Chung-Lu estimate feature
    g_mlp = math.exp(np.mean(np.log(_qerr(est_mlp, T))))
    g_cl = math.exp(np.mean(np.log(_qerr(est_cl, T))))
    print("held-out prefixes: %d, q-error geomean: network %.3g, Chung-Lu %.3g; p90 %.3g vs %.3g" % (
        len(T), g_mlp, g_cl, np.percentile(_qerr(est_mlp, T), 90), np.percentile(_qerr(est_cl, T), 90)))
    assert g_mlp < g_cl


@pytest.mark.parametrize("name", ["4-cycle", "diamond", "house", "5-clique", "4-clique", "6-cycle"])
def test_learned_plans_are_exact(H, name):
    m = H.Model.load(os.path.join(PKG, "mlp_work.npz"))
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    k, e = P.NAMED[name]
    for verify in (False, True):
        order = H.plan(G, k, e, learned=m, verify=verify).info()["order"]
        assert_parity(H, G, g, k, e, order=order)


@pytest.mark.parametrize("cap", [1 << 20, 1 << 26])
def test_learned_plans_choose_segment_rows(H, cap):
    """A learned plan sizes each level's scheduling segment from its model's
    predicted fan-out (enough rows that one segment's predicted output fills the
    next queue once, 2^12..2^22, capped by the level's own queue); an explicit
    chunk_rows overrides it, cost-model plans keep 2^22; every choice counts the
    oracle's matches."""
    from tests.gpu_common import cmp_key, oracle_run

    m = H.Model.load(os.path.join(PKG, "mlp_work.npz"))
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    for name in ["house", "5-clique", "6-cycle", "tailed-triangle"]:
        k, e = P.NAMED[name]
        p = H.plan(G, k, e, learned=m)
        est = p.estimates()
        rows = H.segment_rows(G, p, cap=cap)
        nq = max(0, k - 3)
        qcap = [0] * (H.KMAX + 2)
        for w in range(3, k):
            qcap[w] = max(4096, (cap // nq) // (4 * w))
        for w in range(2, k):
            if w < k - 1 and est[w - 1] > 0 and est[w] > 0:
                want = min(max(4096, int(qcap[w + 1] * est[w - 1] / est[w])), 1 << 22)
            else:
                want = 1 << 22
            if w >= 3:
                want = min(want, qcap[w])
            else:
                want = min(want, g.nnz)
            assert rows[w] == want, (name, cap, w, rows, want)
        assert H.segment_rows(G, p, cap=cap, chunk_rows=5000)[2] == 5000
        cm = H.plan(G, k, e, order=p.info()["order"])
        assert H.segment_rows(G, cm, cap=cap)[2] == min(1 << 22, g.nnz)
        ref = oracle_run(g, k, e)
        for eng in (H.ENGINE_LEVELS, H.ENGINE_GRAPH):
            assert cmp_key(H.count(G, p, cap=cap, engine=eng), k) == cmp_key(ref, k), (name, cap, eng)
        assert cmp_key(H.count_batch(G, [p, cm], cap=cap, engine=H.ENGINE_GRAPH)[0], k) == cmp_key(ref, k)
