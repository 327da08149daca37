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


def test_adam_update_closed_forms():
    """Adam (Kingma and Ba 2015, Algorithm 1) pinned without restating it:
    * constant gradient g: the bias-corrected moments are exactly g and g^2 at
      every step, so each step moves by lr * g / (|g| + eps);
    * g1 = 1 then g2 = -1 (worked by hand): m2 = 0.9*0.1 - 0.1 = -0.01,
      mhat2 = -0.01/0.19; v2 = 0.999*0.001 + 0.001 = 0.001999 = 1 - 0.999^2,
      so vhat2 = 1 and the second step is +lr * 0.01/0.19 / (1 + eps)."""
    lr = 1e-3
    g = np.array([3.0, -0.25, 1e-3, 0.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 6):
        p, m, v = mlp.adam_update(p, m, v, g, t, lr)
        want = -t * lr * g / (np.abs(g) + mlp.EPS)
        np.testing.assert_allclose(p, want, rtol=1e-12, atol=1e-18)
    p, m, v = mlp.adam_update(np.zeros(1), np.zeros(1), np.zeros(1), np.array([1.0]), 1, lr)
    np.testing.assert_allclose(p, [-lr / (1 + mlp.EPS)], rtol=1e-14)
    p, m, v = mlp.adam_update(p, m, v, np.array([-1.0]), 2, lr)
    np.testing.assert_allclose(m, [-0.01], rtol=1e-12)
    np.testing.assert_allclose(v, [0.001999], rtol=1e-12)
    np.testing.assert_allclose(p, [-lr / (1 + mlp.EPS) + lr * (0.01 / 0.19) / (1 + mlp.EPS)], rtol=1e-12)


def test_full_batch_adam_lowers_the_loss_and_matches_its_steps():
    x, y = _data(64, 5)
    p0 = mlp.init(9)
    p, l3 = mlp.adam_full_batch(p0, x, y, 3, 1e-3)
    # the same three steps taken one call at a time
    q, mm, vv = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in (1, 2, 3):
        _, g = mlp.loss_and_grad(q, x, y)
        q, mm, vv = mlp.adam_update(q, mm, vv, g, t, 1e-3)
    np.testing.assert_array_equal(p, q)
    assert l3 < mlp.loss(p0, x, y)
