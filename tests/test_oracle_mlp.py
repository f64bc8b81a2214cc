"""Pins of the warm-start MLP oracle (oracle/mlp.py): the backward pass
against central finite differences of the loss, the first Adam step against
its closed form, the network's trivial cases, the loss mask, and the
invariances of the feature map (rigid motion of body and query together,
periodic images)."""
import numpy as np
import pytest

import workloads
from oracle import mlp


def random_batch(rng, B=16):
    X = rng.normal(0, 0.5, size=(B, mlp.N_IN))
    X[:, 6] = (np.arange(B) % 3 == 0).astype(float)  # both tasks present
    T = rng.normal(0, 0.5, size=(B, mlp.N_OUT))
    return X, T


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    theta = workloads.mlp_init(3) + rng.normal(0, 0.05, size=mlp.P)
    X, T = random_batch(rng)
    g = mlp.grad(theta, X, T)
    idx = np.concatenate([rng.choice(mlp.P, 300, replace=False), np.arange(mlp.P - 260, mlp.P)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, T) - mlp.loss(tm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_first_adam_step_closed_form():
    """With m = v = 0 the bias-corrected moments are g and g^2, so the first
    step is exactly -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    theta = rng.normal(size=mlp.P)
    g = rng.normal(size=mlp.P)
    lr, eps = 1e-3, 1e-8
    t1, m, v = mlp.adam_step(theta, g, np.zeros(mlp.P), np.zeros(mlp.P), 1, lr=lr, eps=eps)
    assert np.allclose(t1, theta - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    theta = np.full(mlp.P, 3.0)
    m = v = np.zeros(mlp.P)
    for t in range(1, 4001):
        theta, m, v = mlp.adam_step(theta, 2 * (theta - 1.0), m, v, t, lr=1e-2)
    assert np.abs(theta - 1.0).max() < 1e-3


def test_zero_weights_give_the_output_bias():
    p = mlp.unpack(np.zeros(mlp.P))
    p["b1"][:] = 0.3
    p["b2"][:] = -0.2
    p["b3"][:] = [0.1, 0.2, 0.3, 0.4]
    X, _ = random_batch(np.random.default_rng(3))
    out, (_, h1, h2) = mlp.forward(mlp.pack(p), X)
    assert np.allclose(out, [0.1, 0.2, 0.3, 0.4], atol=0)
    assert np.allclose(h1, np.tanh(0.3)) and np.allclose(h2, np.tanh(-0.2))


def test_loss_mask_ignores_untargeted_outputs():
    rng = np.random.default_rng(4)
    theta = workloads.mlp_init(5)
    X, T = random_batch(rng)
    T2 = T.copy()
    link = X[:, 6] < 0.5
    T2[link, 1:] += 7.0   # link-fraction rows: only output 0 counts
    T2[~link, 0] -= 5.0   # closest-point rows: only outputs 1..3 count
    assert mlp.loss(theta, X, T) == mlp.loss(theta, X, T2)
    assert np.array_equal(mlp.grad(theta, X, T), mlp.grad(theta, X, T2))


def rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * axis])


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_features_invariant_under_rigid_motion():
    rng = np.random.default_rng(6)
    cpb = rng.normal(0, 2, size=(7, 3))
    k = rng.uniform(5, 15, size=7)
    X, q = np.array([10.0, 11.0, 12.0]), rot([1, 2, 3], 0.7)
    node, e = np.array([14.0, 9.0, 13.0]), np.array([1.0, -1.0, 0.0])
    f0 = mlp.features(cpb, k, X, q, node, e)
    Q = rot([-2, 1, 0.5], 1.1)
    RQ = mlp.quat_matrix(Q)
    shift = np.array([3.0, -4.0, 5.0])
    f1 = mlp.features(cpb, k, RQ @ X + shift, qmul(Q, q), RQ @ node + shift, RQ @ e)
    assert np.allclose(f0, f1, atol=1e-13)
    # periodic image of the query point
    dims = (40, 40, 40)
    f2 = mlp.features(cpb, k, X, q, node + [40, 0, -40], e, dims=dims, periodic=7)
    assert np.allclose(f0, f2, atol=1e-13)


def test_body_block_sorted_normalised_padded():
    cpb = np.array([[1.0, 0, 0], [0, 2.0, 0], [0, 0, 3.0]])
    k = np.array([2.0, 5.0, 2.0])
    blk = mlp.body_block(cpb, k).reshape(20, 4)
    s = 3.0  # sqrt(9)
    assert np.allclose(blk[0], [0, 2 / s, 0, 5 / 9])
    assert np.allclose(blk[1], [1 / s, 0, 0, 2 / 9]) and np.allclose(blk[2], [0, 0, 1.0, 2 / 9])
    assert np.all(blk[3:] == 0)
    assert blk[:, 3].sum() == pytest.approx(1.0)


def test_training_reduces_the_loss():
    rng = np.random.default_rng(8)
    X = rng.normal(0, 0.5, size=(512, mlp.N_IN))
    X[:, 6] = 0.0
    T = np.zeros((512, 4))
    T[:, 0] = 0.5 + 0.3 * np.tanh(X[:, 0] - X[:, 3])
    theta0 = workloads.mlp_init(9)
    l0 = mlp.loss(theta0, X, T)
    theta = mlp.train(theta0, X, T, epochs=20, batch=64, lr=3e-3)
    assert mlp.loss(theta, X, T) < 0.1 * l0
