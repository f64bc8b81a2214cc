"""FP64 oracle of the link-fraction warm start: the feature map, a 3-layer
MLP (87 -> 64 -> 64 -> 4, tanh hidden layers, linear output), its loss,
backward pass and the Adam update.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests and the
benchmark's baseline may use it; the product library never does.

The warm start guesses the root q of C(x_f - s e_i) = 1 (the link fraction
of sec. 2.3.2, found by Newton-Raphson) from the link and the body; the
Newton iteration stays the judge.  Plain numpy in FP64: every layer is
written out as its definition (matrix product, bias, tanh), the backward
pass is the chain rule of that definition, and Adam is the published
update (Kingma & Ba, 2015) with bias correction.

Parameter vector (P = 10052 values), in this order: W1 [87][64], b1 [64],
W2 [64][64], b2 [64], W3 [64][4], b3 [4]; layer l computes
z = h_{l-1} W_l + b_l.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT, MAXCP = 87, 64, 4, 20
SHAPES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))]
P = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def quat_matrix(q):
    """Rotation matrix of a unit quaternion (w, x, y, z): body -> lab."""
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def body_block(cpb, k):
    """The body's 80 constant features: control points in the body frame
    sorted by weight (largest first, ties by index), each (p / s, k / sum k)
    with s = sqrt(sum k), zero-padded to 20 points."""
    cpb = np.asarray(cpb, dtype=np.float64).reshape(-1, 3)
    k = np.asarray(k, dtype=np.float64)
    K = k.sum()
    s = np.sqrt(K)
    order = np.argsort(-k, kind="stable")
    blk = np.zeros((MAXCP, 4))
    blk[:len(k), :3] = cpb[order] / s
    blk[:len(k), 3] = k[order] / K
    return blk.reshape(-1)


def features(cpb, k, X, quat, node, e, dims=None, periodic=0, task=0):
    """87 inputs of one query: the point (the link's fluid node) and the
    direction e in the body frame, the point scaled by 1/sqrt(sum k)
    (minimum image on periodic axes), the task bit (0: link fraction), then
    the body block."""
    R = quat_matrix(np.asarray(quat, dtype=np.float64))
    d = np.asarray(node, dtype=np.float64) - np.asarray(X, dtype=np.float64)
    if dims is not None:
        for a in range(3):
            if (periodic >> a) & 1:
                L = dims[a]
                d[a] -= L * np.floor(d[a] / L + 0.5)
    s = np.sqrt(np.sum(k))
    pb = R.T @ d / s
    eb = R.T @ np.asarray(e, dtype=np.float64)
    return np.concatenate([pb, eb, [float(task)], body_block(cpb, k)])


def forward(theta, X):
    """Outputs [B][4] and the hidden activations (h1, h2)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"] + p["b1"])
    h2 = np.tanh(h1 @ p["W2"] + p["b2"])
    out = h2 @ p["W3"] + p["b3"]
    return out, (X, h1, h2)


def loss_mask(X):
    """Outputs that carry a target: q (output 0) for the link-fraction task,
    the closest-point offset (outputs 1..3) for the other task."""
    X = np.asarray(X, dtype=np.float64)
    m = np.zeros((X.shape[0], N_OUT))
    task = X[:, 6] > 0.5
    m[~task, 0] = 1.0
    m[task, 1:] = 1.0
    return m


def loss(theta, X, T):
    """Mean over the batch of the masked squared error."""
    out, _ = forward(theta, X)
    m = loss_mask(X)
    return float(np.sum(m * (out - T) ** 2) / X.shape[0])


def grad(theta, X, T):
    """Gradient of loss() with respect to theta (chain rule of forward())."""
    p = unpack(theta)
    out, (X, h1, h2) = forward(theta, X)
    B = X.shape[0]
    d_out = 2.0 * loss_mask(X) * (out - T) / B
    g = {"W3": h2.T @ d_out, "b3": d_out.sum(axis=0)}
    d_z2 = (d_out @ p["W3"].T) * (1.0 - h2 ** 2)
    g["W2"] = h1.T @ d_z2
    g["b2"] = d_z2.sum(axis=0)
    d_z1 = (d_z2 @ p["W2"].T) * (1.0 - h1 ** 2)
    g["W1"] = X.T @ d_z1
    g["b1"] = d_z1.sum(axis=0)
    return pack(g)


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, T, epochs=1, batch=256, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, t0=0):
    """Sequential minibatches (the data order as given), Adam per minibatch."""
    theta = np.array(theta, dtype=np.float64)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    t = t0
    n = X.shape[0]
    for _ in range(epochs):
        for a in range(0, n, batch):
            t += 1
            g = grad(theta, X[a:a + batch], T[a:a + batch])
            theta, m, v = adam_step(theta, g, m, v, t, lr, beta1, beta2, eps)
    return theta
