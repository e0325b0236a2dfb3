"""GPU parity of the learned cardinality model's HIP kernels (forward,
backward, Adam) against the FP64 reference evaluated at the same BF16
weights, and exactness of learned plans."""
import numpy as np
import pytest

import graphgen as gg
from graphgen import patterns as P
from oracle import mlp_ref as R
from tests.gpu_common import assert_parity, need_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-3  # max |gpu - ref| / max |ref|: FP32 accumulation over <= 128 + 256 terms


@pytest.fixture(scope="module")
def H():
    return need_gpu()


def _model(H, seed, B):
    rng = np.random.default_rng(seed)
    params = rng.normal(0, 0.08, R.P).astype(np.float32)
    xmean = rng.normal(0, 1, R.F).astype(np.float32)
    xinv = rng.uniform(0.5, 2.0, R.F).astype(np.float32)
    xinv[:5] = 0.0  # constant features are switched off this way
    X = rng.normal(0, 1.5, (B, R.F)).astype(np.float32)
    t = rng.normal(4, 3, B).astype(np.float32)
    m = H.Model().set(params, xmean, xinv, 3.5, 2.25)
    wq = R.bf16_round(params).astype(np.float64)
    return m, params, wq, xmean, xinv, X, t


def _rel(got, ref):
    return float(np.max(np.abs(np.asarray(got, np.float64) - ref)) / max(1e-30, float(np.max(np.abs(ref)))))


@pytest.mark.parametrize("B", [1, 15, 16, 17, 1000, 4099])
def test_forward_matches_reference(H, B):
    m, _, wq, xmean, xinv, X, _ = _model(H, 11 + B, B)
    y = m.forward(X)
    yn, _ = R.forward(wq, xmean, xinv, X)
    assert y.shape == (B,)
    assert _rel(y, yn * 2.25 + 3.5) <= TOL


@pytest.mark.parametrize("B", [1, 33, 1024, 5000])
def test_gradient_matches_reference(H, B):
    m, _, wq, xmean, xinv, X, t = _model(H, 100 + B, B)
    g, loss = m.grad(X, t)
    L, gref = R.loss_and_grad(wq, xmean, xinv, 3.5, 2.25, X, t)
    assert loss == pytest.approx(L, rel=TOL)
    for lo, hi in [(0, R.F * R.H), (R.F * R.H, R.F * R.H + R.H), (R.F * R.H + R.H, R.P - 1), (R.P - 1, R.P)]:
        assert _rel(g[lo:hi], gref[lo:hi]) <= TOL, (lo, hi)


def test_adam_step_matches_reference(H):
    B = 777
    m, params, wq, xmean, xinv, X, t = _model(H, 5, B)
    lr = 1e-3
    losses = m.train(X, t, epochs=1, batch=B, lr=lr, seed=1)  # one full-batch step
    L, gref = R.loss_and_grad(wq, xmean, xinv, 3.5, 2.25, X, t)
    assert losses[0] == pytest.approx(L, rel=TOL)
    wref, _, _ = R.adam_step(params.astype(np.float64), np.zeros(R.P), np.zeros(R.P), gref, 1, lr)
    w = m.get()["params"].astype(np.float64)
    big = np.abs(gref) > 1e-3 * np.abs(gref).max()
    assert big.sum() > R.P // 2
    assert np.max(np.abs(w[big] - wref[big])) <= 1e-6 + TOL * lr
    # every weight moves by at most lr (Adam's first step is lr * g / (|g| + eps))
    assert np.max(np.abs(w - params)) <= lr * (1 + 1e-4)


def test_training_fits_a_smooth_target(H):
    rng = np.random.default_rng(9)
    N = 4096
    X = rng.normal(0, 1, (N, R.F)).astype(np.float32)
    t = (3 + np.tanh(X[:, 0]) * 2 + 0.5 * X[:, 1] ** 2 - X[:, 2] * X[:, 3] * 0.3).astype(np.float32)
    m = H.Model()
    params = (rng.normal(0, 1, R.P) * np.concatenate([np.full(R.F * R.H, np.sqrt(2 / R.F)), np.zeros(R.H),
                                                      np.full(R.H, np.sqrt(1 / R.H)), [0]])).astype(np.float32)
    m.set(params, np.zeros(R.F, np.float32), np.ones(R.F, np.float32), float(t.mean()), float(t.std()))
    losses = m.train(X, t, epochs=60, batch=256, lr=2e-3, seed=3)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.1 * losses[0], losses[[0, -1]]
    pred = m.forward(X)
    assert np.sqrt(np.mean((pred - t) ** 2)) < 0.35 * t.std()


def test_plan_features_layout(H):
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    k, e = P.NAMED["diamond"]
    p = H.plan(G, k, e, order=[1, 2, 0, 3])
    x = H.plan_features(G, p, 3)
    assert x[k - 3] == 1 and x[:6].sum() == 1           # k one-hot
    assert x[6 + 1] == 1 and x[6:13].sum() == 1         # prefix size 3
    assert x[13:41].sum() == 3                          # triangle 1-2-0 in positions
    assert abs(x[86:118].sum() - 1.0) < 1e-5            # degree histogram fractions
    assert np.all(x[69:76][:2] == 1)                    # position 2 joins positions 0 and 1
    with pytest.raises(RuntimeError):
        H.plan_features(G, p, 1)


def test_learned_plan_is_exact(H):
    """Whatever order the (here untrained, random) model picks, the counts are the oracle's."""
    g = gg.chung_lu(3000, 10, 2.3, seed=21)
    G = H.load(g.row_ptr, g.col)
    m, *_ = _model(H, 77, 1)
    for name in ["4-cycle", "diamond", "house", "5-clique", "tailed-triangle"]:
        k, e = P.NAMED[name]
        for verify in (False, True):
            pl = H.plan(G, k, e, learned=m, verify=verify)
            order = pl.info()["order"]
            assert sorted(order) == list(range(k))
            assert_parity(H, G, g, k, e, order=order)
    with pytest.raises(RuntimeError, match="model"):
        H.plan(G, 3, P.NAMED["triangle"][1], learned=True)
