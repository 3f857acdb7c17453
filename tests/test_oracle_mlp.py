"""Pins of the CPU oracle of the learned pruning scorer (float64).

The forward pass, loss and gradients are checked against PyTorch's CPU
autograd in float64 (an independent library implementation of the same
network), against central finite differences, and against closed forms
(a hand-built network with a known output, one Adam step).
"""
import numpy as np
import pytest

from oracle import mlp


def _data(n=257, seed=3):
    rng = np.random.default_rng(seed)
    feats = rng.integers(0, 5000, size=(n, 12))
    feats[:, 5] = 7  # a constant column: its deviation becomes 1
    y = (rng.random(n) < 0.4).astype(np.float64)
    xn, mean, std = mlp.normalize(feats)
    theta = rng.normal(0, 0.3, mlp.NUM_PARAMS)
    return xn, y, theta, feats


def test_parameter_count():
    assert mlp.NUM_PARAMS == 5057


def test_normalize_properties():
    xn, _, _, feats = _data()
    assert np.allclose(xn[:, [0, 1, 2, 3, 4, 6]].mean(axis=0), 0.0, atol=1e-12)
    assert np.allclose(xn[:, [0, 1, 2, 3, 4, 6]].std(axis=0), 1.0, atol=1e-12)
    assert np.allclose(xn[:, 5], 0.0)
    # the same statistics applied to new data
    xn2, _, _ = mlp.normalize(feats[:10], *mlp.normalize(feats)[1:])
    assert np.allclose(xn2, xn[:10])


def test_against_torch_autograd():
    torch = pytest.importorskip("torch")
    xn, y, theta, _ = _data()
    L, g = mlp.grad(theta, xn, y)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    o, parts = 0, []
    for s in mlp.SIZES:
        n = int(np.prod(s))
        parts.append(t[o:o + n].reshape(s))
        o += n
    W1, b1, W2, b2, W3, b3 = parts
    X = torch.tensor(xn, dtype=torch.float64)
    h1 = torch.relu(X @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    z = (h2 @ W3.T + b3)[:, 0]
    Lt = torch.nn.functional.binary_cross_entropy_with_logits(
        z, torch.tensor(y, dtype=torch.float64))
    Lt.backward()
    assert abs(L - Lt.item()) <= 1e-12 * max(1.0, abs(L))
    gt = t.grad.numpy()
    assert np.allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_finite_differences():
    xn, y, theta, _ = _data(n=64, seed=5)
    _, g = mlp.grad(theta, xn, y)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.NUM_PARAMS, 300, replace=False),
                          [0, 767, 768, 831, 832, 4927, 4928, 4991, 4992, 5056]])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, xn, y) - mlp.loss(tm, xn, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, i


def test_closed_form_absolute_value():
    """W1 rows 0 and 1 pick +x3 and -x3, W2 = identity, W3 sums units 0
    and 1: the logit is |x3|."""
    theta = np.zeros(mlp.NUM_PARAMS)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta)
    W1[0, 3] = 1.0
    W1[1, 3] = -1.0
    W2[:, :] = np.eye(64)
    W3[0, 0] = W3[0, 1] = 1.0
    x = np.random.default_rng(2).normal(size=(50, 12))
    z, _ = mlp.forward(theta, x)
    assert np.allclose(z, np.abs(x[:, 3]))
    y = np.ones(50)
    assert abs(mlp.loss(theta, x, y) - np.mean(np.log1p(np.exp(-np.abs(x[:, 3]))))) < 1e-12


def test_closed_form_constant_output():
    """All weights zero, b3 = c: loss = softplus(c) - mean(y) c and the
    gradient is sigmoid(c) - mean(y) on b3 only."""
    theta = np.zeros(mlp.NUM_PARAMS)
    theta[-1] = 0.7
    xn, y, _, _ = _data()
    L, g = mlp.grad(theta, xn, y)
    assert abs(L - (np.log1p(np.exp(0.7)) - y.mean() * 0.7)) < 1e-12
    assert abs(g[-1] - (1 / (1 + np.exp(-0.7)) - y.mean())) < 1e-12
    assert np.all(g[:-1] == 0)


def test_adam_first_step():
    """First Adam step: m_hat = g, v_hat = g^2, so theta moves by
    -lr g / (|g| + eps)."""
    xn, y, theta, _ = _data()
    _, g = mlp.grad(theta, xn, y)
    t1, losses = mlp.adam(theta, xn, y, 1, lr=1e-3)
    assert np.allclose(t1 - theta, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    assert losses[0] == mlp.loss(theta, xn, y)


def test_adam_decreases_loss_and_threshold():
    xn, y, theta, _ = _data(n=300, seed=9)
    theta = theta * 0.1
    t, losses = mlp.adam(theta, xn, y, 300, lr=1e-2)
    assert losses[-1] < losses[0]
    p = mlp.predict(t, xn)
    th = mlp.threshold_zero_miss(p, y)
    assert not np.any((p < th) & (y == 1))
    assert np.any(p[y == 1] == th)
