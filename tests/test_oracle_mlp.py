"""Pins for the cost-model oracle: finite differences, Adam's first-step closed form,
degenerate networks and the feature vector on a hand-checked example."""
import math

import numpy as np
import pytest

from oracle import mlp, features


def _params(rng, f=17, h1=64, h2=64):
    return {
        "W1": rng.normal(0, math.sqrt(2 / f), (h1, f)), "b1": rng.normal(0, 0.1, h1),
        "W2": rng.normal(0, math.sqrt(2 / h1), (h2, h1)), "b2": rng.normal(0, 0.1, h2),
        "W3": rng.normal(0, math.sqrt(2 / h2), (1, h2)), "b3": rng.normal(0, 0.1, 1),
    }


def test_gradients_match_central_differences():
    rng = np.random.default_rng(20)
    p = _params(rng, f=7, h1=9, h2=5)
    X = rng.normal(size=(12, 7))
    y = rng.normal(size=12)
    mask = (rng.uniform(size=12) < 0.8).astype(np.float64)
    out, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, out, y, mask)
    h = 1e-6
    for k in mlp.PARAM_ORDER:
        flat = p[k].reshape(-1)
        gk = g[k].reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(p, X)[0], y, mask)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(p, X)[0], y, mask)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gk[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, gk[idx])


def test_zero_network_outputs_bias_and_loss():
    p = {k: np.zeros_like(v) for k, v in _params(np.random.default_rng(0)).items()}
    p["b3"] = np.array([0.75])
    X = np.random.default_rng(1).normal(size=(5, 17))
    out, _ = mlp.forward(p, X)
    assert np.all(out == 0.75)
    y = np.array([0.75, 1.75, 0.75, -0.25, 0.75])
    assert mlp.loss(out, y, np.ones(5)) == pytest.approx((1 + 1) / 5)
    assert mlp.loss(out, y, np.array([1, 0, 1, 0, 1.0])) == 0.0


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(21)
    p = _params(rng)
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    z = mlp.zeros_like(p)
    p1, m1, v1 = mlp.adam_step(p, g, z, z, 1, lr=1e-3, eps=1e-8)
    for k in mlp.PARAM_ORDER:
        # m_hat = g, v_hat = g^2 at t = 1
        want = p[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(p1[k], want, rtol=0, atol=1e-15)
        assert np.allclose(m1[k], 0.1 * g[k]) and np.allclose(v1[k], 0.001 * g[k] ** 2)


def test_training_reduces_loss_on_a_linear_target():
    rng = np.random.default_rng(22)
    X = rng.normal(size=(512, 17))
    w = rng.normal(size=17)
    y = X @ w * 0.1
    p = _params(rng)
    batches = [rng.integers(0, 512, 64) for _ in range(300)]
    _, losses = mlp.train(p, X, y, np.ones(512), batches, lr=3e-3)
    assert np.mean(losses[-20:]) < 0.25 * np.mean(losses[:20])


def test_features_hand_example():
    # 2*A + B % C - trans(D): 5 operator entries, 4 operands, 1 trans, fp32, 4096 x 4096, per-row sum
    postfix = [("scalar", 0), ("load", 0), ("schur",), ("load", 1), ("load", 2), ("schur",), ("add",),
               ("load", 3), ("trans",), ("sub",)]
    f = features.features(postfix, "f32", 4096, 4096, "dim1", (4, 2, 4, 8))
    assert f.shape == (features.N_FEATURES,)
    # tiled: 64 x 64 = 4096 tiles, capped at 8 * 256 = 2048 workgroups of 256 threads, 32 elements each
    want = [5, 4, 0, 0, 1, 0, math.log2(4097), math.log2(4097), 1, 0, 0, 0, 1, 2, 1, 2, 3,
            math.log2(1 + 4096 * 4096), 1, 11, math.log2(33), 6, 6]
    assert np.allclose(f, want)
    # the same with 128 x 32 tiles: 32 x 128 = 4096 tiles, again capped at 2048 workgroups
    f = features.features(postfix, "f32", 4096, 4096, "dim1", (4, 1, 4, 8, 128, 32))
    want[14] = 0                 # log2(ept = 1)
    want[21:] = [7, 5]
    assert np.allclose(f, want)
    # 256 x 16 tiles on 300 x 50: 2 x 4 = 8 tiles (below the cap), 15000 / 2048 elements per thread
    f = features.features(postfix, "f32", 300, 50, "none", (2, 1, 4, 16, 256, 16))
    assert np.allclose(f[17:], [math.log2(15001), 1, 3, math.log2(1 + 15000 / 2048), 8, 4])
    # exp(A) / (1 + abs(B)) on 1000 x 3, element-wise: flat, 750 groups of 4 fit one workgroup of
    # 256 threads x 4 groups; 3000 / 256 elements per thread
    wpost = [("load", 0), ("exp",), ("scalar", 0), ("load", 1), ("abs",), ("add",), ("div",)]
    f = features.features(wpost, "f32", 1000, 3, "none", (4, 4, 4, 8))
    want = [4, 2, 0, 0, 1, 0, math.log2(1001), 2, 0, 1, 0, 0, 0, 2, 2, 2, 3,
            math.log2(3001), 0, 0, math.log2(1 + 3000 / 256), 0, 0]
    assert np.allclose(f, want)


def test_transposed_leaf_detection():
    A, B = ("load", 0), ("load", 1)
    assert not features.has_transposed_leaf([A, ("trans",), ("trans",), B, ("add",)])
    assert features.has_transposed_leaf([A, B, ("trans",), ("add",), ("trans",)])     # A under one trans
    assert not features.has_transposed_leaf([A, ("trans",), ("neg",), ("trans",)])
    assert features.has_transposed_leaf([("scalar", 0), A, ("trans",), ("schur",)])
