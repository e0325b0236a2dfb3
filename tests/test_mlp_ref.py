"""Pins of the FP64 MLP reference (oracle/mlp_ref.py) against facts other than
itself: central finite differences, a network small enough to evaluate by
hand, torch's own BF16 rounding, and the closed form of Adam's first step."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as R


def _rand_model(rng, scale=0.1):
    params = rng.normal(0, scale, R.P)
    xmean = rng.normal(0, 1, R.F)
    xinv = rng.uniform(0.5, 2.0, R.F)
    return params, xmean, xinv


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    params, xmean, xinv = _rand_model(rng)
    X = rng.normal(0, 1, (12, R.F))
    t = rng.normal(3, 2, 12)
    tmean, tstd = 2.5, 1.7
    L, g = R.loss_and_grad(params, xmean, xinv, tmean, tstd, X, t)
    assert L == pytest.approx(R.loss(params, xmean, xinv, tmean, tstd, X, t), rel=1e-14)
    # coordinates in every block: W1, b1, W2, b2
    idx = list(rng.choice(R.F * R.H, 40, replace=False)) + list(R.F * R.H + rng.choice(R.H, 10, replace=False)) + \
        list(R.F * R.H + R.H + rng.choice(R.H, 10, replace=False)) + [R.P - 1]
    h = 1e-6
    for i in idx:
        e = np.zeros(R.P)
        e[i] = h
        num = (R.loss(params + e, xmean, xinv, tmean, tstd, X, t) -
               R.loss(params - e, xmean, xinv, tmean, tstd, X, t)) / (2 * h)
        assert num == pytest.approx(g[i], rel=1e-5, abs=1e-9), i


def test_forward_by_hand():
    # two live hidden units: h0 = relu(2*xn0 + 1), h1 = relu(-xn1 + 0.5); y = 3*h0 - 2*h1 + 0.25
    W1 = np.zeros((R.F, R.H))
    b1 = np.full(R.H, -1.0)  # every other unit is dead for inputs of 0
    W1[0, 0], b1[0] = 2.0, 1.0
    W1[1, 1], b1[1] = -1.0, 0.5
    W2 = np.zeros(R.H)
    W2[0], W2[1] = 3.0, -2.0
    params = R.pack(W1, b1, W2, 0.25)
    X = np.zeros((3, R.F))
    X[0, 0], X[0, 1] = 1.0, 0.0    # h0 = 3, h1 = 0.5  -> 9 - 1 + 0.25
    X[1, 0], X[1, 1] = -1.0, 2.0   # h0 = 0, h1 = 0    -> 0.25
    X[2, 0], X[2, 1] = 0.5, -1.5   # h0 = 2, h1 = 2    -> 6 - 4 + 0.25
    yn, _ = R.forward(params, np.zeros(R.F), np.ones(R.F), X)
    assert yn.tolist() == [8.25, 0.25, 2.25]
    # standardisation of the inputs: x = 2*xn + 5
    yn2, _ = R.forward(params, np.full(R.F, 5.0), np.full(R.F, 0.5), 2 * X + 5)
    assert np.allclose(yn2, yn)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000),
                        [0.0, -0.0, np.inf, -np.inf, 1.0, 65504.0, 3.0e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = R.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    # exact ties round to the even kept part
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000], dtype=np.uint32).view(np.float32)
    assert R.bf16_round(ties).view(np.uint32).tolist() == [0x3F800000, 0x3F820000, 0xBF800000]
    assert np.isnan(R.bf16_round(np.array([np.nan], np.float32)))[0]


def test_adam_first_step_closed_form():
    # at step 1, m_hat = g and v_hat = g^2, so the update is lr * g / (|g| + eps)
    rng = np.random.default_rng(5)
    w = rng.normal(0, 1, 100)
    g = rng.normal(0, 1, 100)
    w1, m1, v1 = R.adam_step(w, np.zeros(100), np.zeros(100), g, 1, 1e-3, eps=1e-8)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
