"""Test infrastructure: a plain FP64 reference of the learned cost model.

Only the tests (and nothing on the product path) use this module.  It shares
no code with the library's HIP kernels.

Model (the estimator slot of the optimiser, Section 3.3, left open by the
paper; it predicts the log of a per-step size of a matching order): a
2-layer MLP with F = 128 inputs, H = 256 ReLU hidden units and one output,
    xn  = (x - xmean) * xinv
    z   = xn @ W1 + b1          (W1 is F x H)
    yn  = relu(z) @ W2 + b2
    label = yn * tstd + tmean   (the predicted log-size)
Parameters are packed as W1 (row-major, F x H) | b1 (H) | W2 (H) | b2 (1).
The loss is L = mean((yn - (t - tmean) / tstd)^2).  The library computes with
BF16 copies of FP32 master weights: `bf16_round` gives the values it uses, so
the reference is evaluated at those.
"""
from __future__ import annotations

import numpy as np

F, H = 128, 256
P = F * H + 2 * H + 1


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.shape == (P,)
    W1 = p[: F * H].reshape(F, H)
    b1 = p[F * H: F * H + H]
    W2 = p[F * H + H: F * H + 2 * H]
    b2 = p[F * H + 2 * H]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2):
    return np.concatenate([np.asarray(W1, np.float64).reshape(-1), np.asarray(b1, np.float64),
                           np.asarray(W2, np.float64), np.asarray([b2], np.float64)])


def bf16_round(x):
    """FP32 -> BF16 -> FP32, round to nearest with ties to even (NaN kept)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    upper = u >> 16
    lower = u & 0xFFFF
    # round up when the dropped half is above the midpoint, or at the midpoint with an odd kept part
    up = (lower > 0x8000) | ((lower == 0x8000) & ((upper & 1) == 1))
    r = (upper + up.astype(np.uint64)) << 16
    nan = np.isnan(a)
    r = np.where(nan, (u | 0x400000) & 0xFFFF0000, r)
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def forward(params, xmean, xinv, X):
    """Returns (yn, z) for inputs X (B x F), in FP64."""
    W1, b1, W2, b2 = unpack(params)
    X = np.asarray(X, dtype=np.float64).reshape(-1, F)
    xn = (X - np.asarray(xmean, np.float64)) * np.asarray(xinv, np.float64)
    z = xn @ W1 + b1
    yn = np.maximum(z, 0.0) @ W2 + b2
    return yn, z


def loss(params, xmean, xinv, tmean, tstd, X, t):
    yn, _ = forward(params, xmean, xinv, X)
    tn = (np.asarray(t, np.float64) - tmean) / tstd
    return float(np.mean((yn - tn) ** 2))


def loss_and_grad(params, xmean, xinv, tmean, tstd, X, t):
    """Loss and its gradient with respect to the packed parameters (chain rule, FP64)."""
    W1, b1, W2, b2 = unpack(params)
    X = np.asarray(X, dtype=np.float64).reshape(-1, F)
    B = X.shape[0]
    xn = (X - np.asarray(xmean, np.float64)) * np.asarray(xinv, np.float64)
    z = xn @ W1 + b1
    a = np.maximum(z, 0.0)
    yn = a @ W2 + b2
    tn = (np.asarray(t, np.float64) - tmean) / tstd
    d = yn - tn
    L = float(np.mean(d ** 2))
    g = 2.0 * d / B                      # dL/dyn
    gW2 = a.T @ g
    gb2 = g.sum()
    dz = np.outer(g, W2) * (z > 0)       # dL/dz
    gW1 = xn.T @ dz
    gb1 = dz.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2)


def adam_step(w, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; `step` counts from 1."""
    w, m, v, g = (np.asarray(a, np.float64) for a in (w, m, v, g))
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
