"""Float64 oracle of the scheduler's cost model.

TEST INFRASTRUCTURE ONLY: used by tests/, never by the library.

The paper describes no scheduler: this cost model is a project addition that
orders the miner's work, never its results.  It is a small perceptron that
maps per-task features to a predicted cost; its weights are stored in BF16 and
it is trained on the device.  This module restates that network in
plain numpy float64 so the device forward pass, the hand-written backward pass
and the Adam update can be compared against it:

  * x_n = (x - mean) * inv_std                      (input standardisation)
  * h1  = relu(x_n W1 + b1),  W1: 8 x 64
  * h2  = relu(h1 W2 + b2),   W2: 64 x 64
  * f   = h2 . W3 + b3,       W3: 64
  * L   = scale * sum_r (f_r - y_r)^2

Parameters are one flat vector in the order W1 (row-major, [in][out]), b1,
W2, b2, W3, b3 -- 4,801 values.  The device keeps an FP32 master copy and
computes with the master rounded to BF16 (round to nearest, ties to even on
the upper 16 bits of the FP32 pattern); `bf16_round` is that rounding.

Pins (tests/test_oracle_mlp.py): the backward pass against central finite
differences of the forward pass; the forward pass of an all-active network
against the product of its weight matrices (it is then affine); a dead first
layer against its constant output; BF16 rounding against values fixed by the
format's definition; Adam against closed forms: the first step is -lr sign(g),
a constant gradient moves every step by -lr sign(g), and a hand-computed
two-step sequence with a sign change (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

IN, H = 8, 64
W1, B1 = 0, IN * H
W2 = B1 + H
B2 = W2 + H * H
W3 = B2 + H
B3 = W3 + H
PARAMS = B3 + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (PARAMS,)
    return (p[W1:B1].reshape(IN, H), p[B1:W2], p[W2:B2].reshape(H, H), p[B2:W3], p[W3:B3],
            float(p[B3]))


def pack(w1, b1, w2, b2, w3, b3):
    return np.concatenate([np.ravel(w1), b1, np.ravel(w2), b2, w3, [b3]]).astype(np.float64)


def bf16_round(x):
    """float32 values rounded to the nearest BF16 (ties to even), as float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def standardise(X, norm):
    X = np.asarray(X, dtype=np.float64)
    norm = np.asarray(norm, dtype=np.float64)
    return (X - norm[:IN]) * norm[IN:2 * IN]


def forward(p, norm, X):
    """Predictions f (rows,) and the activations the backward pass needs."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    xn = standardise(X, norm)
    z1 = xn @ w1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w2 + b2
    h2 = np.maximum(z2, 0.0)
    f = h2 @ w3 + b3
    return f, (xn, z1, h1, z2, h2)


def loss(p, norm, X, Y, scale):
    f, _ = forward(p, norm, X)
    return scale * float(np.sum((f - np.asarray(Y, dtype=np.float64)) ** 2))


def grad(p, norm, X, Y, scale):
    """Gradient of `loss` with respect to the flat parameter vector."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    f, (xn, z1, h1, z2, h2) = forward(p, norm, X)
    d_f = 2.0 * scale * (f - np.asarray(Y, dtype=np.float64))  # dL/df
    g_w3 = h2.T @ d_f
    g_b3 = float(np.sum(d_f))
    d_z2 = np.outer(d_f, w3) * (z2 > 0)
    g_w2 = h1.T @ d_z2
    g_b2 = d_z2.sum(axis=0)
    d_z1 = (d_z2 @ w2.T) * (z1 > 0)
    g_w1 = xn.T @ d_z1
    g_b1 = d_z1.sum(axis=0)
    return pack(g_w1, g_b1, g_w2, g_b2, g_w3, g_b3)


def adam(master, m, v, g, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) with bias correction."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v


def label(cost):
    """Training target of a subtree task: log2(1 + its cost), the cost being the
    64-bit column words the depth-first evaluation of its subtree streams."""
    return np.log2(1.0 + np.asarray(cost, dtype=np.float64))
