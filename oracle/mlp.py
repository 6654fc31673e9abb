"""Binary64 reference of the launch-configuration cost model (test infrastructure only).

The paper has no learned component; this network is the reading of the learned
tuner chosen for the fused path (a reading of ours):

    h1  = relu(X W1^T + b1)          W1: H1 x F
    h2  = relu(h1 W2^T + b2)         W2: H2 x H1
    out = h2 W3^T + b3               W3: 1 x H2
    L   = sum_i m_i (out_i - y_i)^2 / sum_i m_i        (masked mean squared error)

trained with Adam (bias-corrected first and second moments).  relu'(0) = 0.
Parameters are a dict of float64 arrays: W1 b1 W2 b2 W3 b3.  Parity: the analytic
gradients are pinned against central finite differences; Adam against its
first-step closed form.
"""
from __future__ import annotations

import numpy as np

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(p: dict, X: np.ndarray):
    """Returns (out[B], cache) in binary64."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = (h2 @ p["W3"].T + p["b3"]).reshape(-1)
    return out, (X, z1, h1, z2, h2)


def loss(out: np.ndarray, y: np.ndarray, mask: np.ndarray) -> float:
    m = np.asarray(mask, dtype=np.float64)
    d = np.asarray(out, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    cnt = m.sum()
    return float((m * d * d).sum() / cnt) if cnt > 0 else 0.0


def backward(p: dict, cache, out, y, mask) -> dict:
    """Gradients of `loss` with respect to every parameter."""
    X, z1, h1, z2, h2 = cache
    m = np.asarray(mask, dtype=np.float64)
    cnt = m.sum()
    g_out = (2.0 * m * (np.asarray(out) - np.asarray(y, dtype=np.float64)) / cnt) if cnt > 0 else np.zeros_like(out)
    g_out = g_out.reshape(-1, 1)
    g = {}
    g["W3"] = g_out.T @ h2
    g["b3"] = g_out.sum(axis=0)
    g_h2 = g_out @ p["W3"]
    g_z2 = g_h2 * (z2 > 0)
    g["W2"] = g_z2.T @ h1
    g["b2"] = g_z2.sum(axis=0)
    g_h1 = g_z2 @ p["W2"]
    g_z1 = g_h1 * (z1 > 0)
    g["W1"] = g_z1.T @ X
    g["b1"] = g_z1.sum(axis=0)
    return g


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (t starts at 1); returns new (p, m, v)."""
    np_, nm, nv = {}, {}, {}
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for k in PARAM_ORDER:
        nm[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        nv[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mhat = nm[k] / c1
        vhat = nv[k] / c2
        np_[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return np_, nm, nv


def zeros_like(p: dict) -> dict:
    return {k: np.zeros_like(np.asarray(p[k], dtype=np.float64)) for k in PARAM_ORDER}


def train(p: dict, X, y, mask, batches, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Plain Adam over a list of index batches (each an int array into X); returns (p, losses)."""
    p = {k: np.asarray(v, dtype=np.float64).copy() for k, v in p.items()}
    m = zeros_like(p)
    v = zeros_like(p)
    losses = []
    for t, idx in enumerate(batches, start=1):
        out, cache = forward(p, X[idx])
        losses.append(loss(out, y[idx], mask[idx]))
        g = backward(p, cache, out, y[idx], mask[idx])
        p, m, v = adam_step(p, g, m, v, t, lr, beta1, beta2, eps)
    return p, losses
