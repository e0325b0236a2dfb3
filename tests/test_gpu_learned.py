"""What the trained networks gain over the method without them.

* Cardinality: on graphs and patterns held out of training (new seeds, a
  smaller Chung-Lu graph and an R-MAT graph), the cardinality network's
  estimates of |R(prefix)| -- the quantity the cost model of the optimiser
  ranks orders by -- have a much smaller q-error than the Chung-Lu estimator
  the plain cost model uses.  True sizes are exact whole-graph counts of
  prefix plans.
* Planning: plans chosen by the work network (with measured verification)
  count exactly the same matches as the cost model's plans and the oracle.
"""
import math
import os
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


def test_count_model_beats_chung_lu_on_held_out_graphs(H):
    m = H.Model.load(os.path.join(PKG, "mlp_count.npz"))
    pats = P.random_patterns(24, seed=4242, kmin=4, kmax=6, distinct="labelled")
    X, T = [], []
    for g in [gg.chung_lu(200_000, 16, 2.4, seed=99), gg.rmat(17, 16, seed=99)]:
        G = H.load(g.row_ptr, g.col)
        deadline = time.time() + 35
        for q in pats:
            if time.time() > deadline:
                break
            p = H.plan(G, q["k"], q["edges"])
            for s in range(2, q["k"] + 1):
                r = H.count(G, H.plan_prefix(p, s), work_limit=int(3e8), hash=False)
                if r["stopped"]:
                    break  # deeper prefixes cost more
                X.append(H.plan_features(G, p, s))
                T.append(float(r["count"]))
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
    assert g_mlp < 0.5 * g_cl


@pytest.mark.parametrize("name", ["4-cycle", "diamond", "house", "5-clique", "4-clique", "6-cycle"])
def test_learned_plans_are_exact(H, name):
    m = H.Model.load(os.path.join(PKG, "mlp_work.npz"))
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    k, e = P.NAMED[name]
    for verify in (False, True):
        order = H.plan(G, k, e, learned=m, verify=verify).info()["order"]
        assert_parity(H, G, g, k, e, order=order)
