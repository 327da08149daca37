"""Pins of the FP64 MLP oracle: analytic gradients equal central finite
differences; a zero-weight network has the closed-form gradient of its bias;
training drives the loss down on a learnable target."""
import numpy as np

from oracle import mlp


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.integers(0, 17, n), rng.integers(0, 17, n), rng.integers(0, 17, n),
                         rng.integers(0, 7, n), rng.integers(0, 3, n), rng.integers(0, 3, n),
                         rng.integers(0, 3, n), rng.integers(0, 2, n)]).astype(np.float64)
    y = 0.5 * x[:, 0] + 0.4 * x[:, 1] + 0.3 * x[:, 2] - 8 + 0.2 * x[:, 4]
    return x, y


def test_gradient_matches_finite_differences():
    x, y = _data(64, 1)
    p = mlp.init(3)
    p[mlp.SIZES[0]:mlp.SIZES[0] + mlp.H] = 0.1   # positive biases keep units active
    _, g = mlp.loss_and_grad(p, x, y)
    rng = np.random.default_rng(2)
    which = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [mlp.N_PARAMS - 1]])
    num = mlp.numeric_grad(p, x, y, which)
    np.testing.assert_allclose(g[which], num, rtol=1e-5, atol=1e-7)


def test_zero_network_bias_gradient_closed_form():
    x, y = _data(32, 4)
    p = np.zeros(mlp.N_PARAMS)
    l, g = mlp.loss_and_grad(p, x, y)
    # out = 0 everywhere: L = mean(y^2), dL/db3 = -2 mean(y), every other gradient 0
    assert abs(l - np.mean(y ** 2)) < 1e-12
    assert abs(g[-1] + 2 * np.mean(y)) < 1e-12
    assert np.all(g[:-1] == 0)


def test_training_reduces_loss():
    x, y = _data(512, 5)
    p0 = mlp.init(7)
    p = mlp.adam_train(x, y, epochs=30, batch=64, lr=3e-3, seed=7)
    assert mlp.loss(p, x, y) < 0.05 * mlp.loss(p0, x, y)
