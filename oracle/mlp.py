"""CPU oracle of the learned pruning scorer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP
library.

A multilayer perceptron 12 -> 64 -> 64 -> 1 with ReLU hidden units scores a
block-pair flow problem by the probability (sigmoid of the output) that
refining it improves the cut; it is trained with the mean binary
cross-entropy on logits and full-batch Adam.  Everything here is float64.

Parameter vector layout (5,057 values, row-major matrices):
    W1 [64 x 12], b1 [64], W2 [64 x 64], b2 [64], W3 [1 x 64], b3 [1]
Features: 12 non-negative integers per problem, transformed by log1p and
z-scored with the training set's mean and population standard deviation
(a deviation below 1e-9, i.e. a constant column up to rounding, is
replaced by 1).

The paper prunes refinements with fixed rules (section "Parallel Active
Block Scheduling", paragraph "Implementation Details": skip pairs whose
cut is small); the scorer replaces that rule and is judged only by the
missed improvement of the problems it skips.
"""
from __future__ import annotations

import numpy as np

SIZES = [(64, 12), (64,), (64, 64), (64,), (1, 64), (1,)]
NUM_PARAMS = sum(int(np.prod(s)) for s in SIZES)  # 5057


def unpack(theta):
    """Views (W1, b1, W2, b2, W3, b3) of a flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def normalize(features, mean=None, std=None):
    """log1p then z-score; returns (normalized, mean, std)."""
    f = np.log1p(np.asarray(features, dtype=np.float64))
    if mean is None:
        mean = f.mean(axis=0)
        std = f.std(axis=0)
        std = np.where(std > 1e-9, std, 1.0)
    return (f - mean) / std, mean, std


def forward(theta, xn):
    """Logits of the normalized samples xn [N x 12], and the hidden layers."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = xn @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z = (h2 @ W3.T + b3)[:, 0]
    return z, (z1, h1, z2, h2)


def loss(theta, xn, y):
    """Mean binary cross-entropy on logits: softplus(z) - y z."""
    z, _ = forward(theta, xn)
    return float(np.mean(np.logaddexp(0.0, z) - np.asarray(y, dtype=np.float64) * z))


def grad(theta, xn, y):
    """(loss, gradient) by the chain rule through the three layers."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y = np.asarray(y, dtype=np.float64)
    n = xn.shape[0]
    z, (z1, h1, z2, h2) = forward(theta, xn)
    L = float(np.mean(np.logaddexp(0.0, z) - y * z))
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n            # dL/dz        [N]
    gW3 = dz[None, :] @ h2                              # [1 x 64]
    gb3 = np.array([dz.sum()])
    dh2 = dz[:, None] * W3                              # [N x 64]
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1                                    # [64 x 64]
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ xn                                    # [64 x 12]
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam(theta, xn, y, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Full-batch Adam (Kingma and Ba); returns (theta, losses per step)."""
    theta = np.array(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for t in range(1, steps + 1):
        L, g = grad(theta, xn, y)
        losses.append(L)
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, losses


def predict(theta, xn):
    z, _ = forward(theta, xn)
    return 1.0 / (1.0 + np.exp(-z))


def threshold_zero_miss(p, y):
    """Largest threshold theta such that skipping every problem scored below
    it skips no positive one: the smallest score of a positive (1.0 if there
    is no positive)."""
    p = np.asarray(p, dtype=np.float64)
    y = np.asarray(y).astype(bool)
    return float(p[y].min()) if y.any() else 1.0
