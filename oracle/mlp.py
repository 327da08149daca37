"""FP64 oracle of the step-cost MLP (test infrastructure only).

Architecture (the model's definition): inputs x (8 features) are scaled
elementwise by IN_SCALE, then h1 = relu(W1 xs + b1) (128), h2 = relu(W2 h1 + b2)
(128), out = W3 h2 + b3 (1).  Loss: mean over rows of (out - y)^2.
Parameter vector order: W1 [128][8], b1, W2 [128][128], b2, W3 [1][128], b3.
``loss_and_grad`` is reverse-mode differentiation written out by hand;
``numeric_grad`` is central finite differences (the pin).  ``adam_update`` is
one step of Adam (Kingma and Ba, 2015), pinned by closed forms: under a
constant gradient the bias-corrected moments equal g and g^2 exactly, and a
two-step case is worked by hand.
"""
from __future__ import annotations

import numpy as np

F, H = 8, 128
IN_SCALE = np.array([1 / 16, 1 / 16, 1 / 16, 1 / 8, 1 / 3, 1 / 3, 1 / 2, 1.0])
SIZES = [H * F, H, H * H, H, H, 1]
N_PARAMS = sum(SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for s in SIZES:
        out.append(p[o:o + s])
        o += s
    w1, b1, w2, b2, w3, b3 = out
    return w1.reshape(H, F), b1, w2.reshape(H, H), b2, w3.reshape(1, H), b3


def forward(p, x):
    w1, b1, w2, b2, w3, b3 = unpack(p)
    xs = np.asarray(x, np.float64) * IN_SCALE
    a1 = xs @ w1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w2.T + b2
    h2 = np.maximum(a2, 0.0)
    out = (h2 @ w3.T + b3)[:, 0]
    return out, (xs, a1, h1, a2, h2)


def loss(p, x, y):
    out, _ = forward(p, x)
    return float(np.mean((out - np.asarray(y, np.float64)) ** 2))


def loss_and_grad(p, x, y):
    w1, b1, w2, b2, w3, b3 = unpack(p)
    out, (xs, a1, h1, a2, h2) = forward(p, x)
    n = len(out)
    d_out = 2.0 * (out - np.asarray(y, np.float64)) / n          # dL/dout
    g_w3 = d_out[None, :] @ h2                                    # (1, H)
    g_b3 = np.array([d_out.sum()])
    d_a2 = (d_out[:, None] * w3) * (a2 > 0)                       # (n, H)
    g_w2 = d_a2.T @ h1
    g_b2 = d_a2.sum(axis=0)
    d_a1 = (d_a2 @ w2) * (a1 > 0)
    g_w1 = d_a1.T @ xs
    g_b1 = d_a1.sum(axis=0)
    g = np.concatenate([g_w1.ravel(), g_b1, g_w2.ravel(), g_b2, g_w3.ravel(), g_b3])
    return float(np.mean((out - np.asarray(y, np.float64)) ** 2)), g


def numeric_grad(p, x, y, which, h=1e-6):
    p = np.array(p, dtype=np.float64)
    g = np.zeros(len(which))
    for t, i in enumerate(which):
        q = p.copy()
        q[i] += h
        lp = loss(q, x, y)
        q[i] -= 2 * h
        lm = loss(q, x, y)
        g[t] = (lp - lm) / (2 * h)
    return g


def init(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for s, fan_in in zip(SIZES, [F, None, H, None, H, None]):
        if fan_in is None:
            parts.append(np.zeros(s))
        else:
            b = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-b, b, size=s))
    return np.concatenate(parts)


BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def adam_update(p, m, v, g, t, lr):
    """One Adam step (Kingma and Ba, Algorithm 1): first and second moment
    averages, their bias corrections at step t (1-based), and the update
    p - lr * mhat / (sqrt(vhat) + eps).  Returns the new (p, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mhat = m / (1.0 - BETA1 ** t)
    vhat = v / (1.0 - BETA2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + EPS), m, v


def adam_full_batch(p0, x, y, steps, lr):
    """`steps` Adam steps on all rows from p0 and zero moments; returns
    (parameters, loss after the last step)."""
    p = np.array(p0, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, steps + 1):
        _, g = loss_and_grad(p, x, y)
        p, m, v = adam_update(p, m, v, g, t, lr)
    return p, loss(p, x, y)


def adam_train(x, y, epochs, batch, lr, seed):
    """Plain FP64 minibatch Adam, for timing beside the device trainer."""
    p = init(seed)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    rng = np.random.default_rng(seed + 1)
    t = 0
    n = len(y)
    for _ in range(epochs):
        order = rng.permutation(n)
        for r0 in range(0, n, batch):
            idx = order[r0:r0 + batch]
            _, g = loss_and_grad(p, x[idx], y[idx])
            t += 1
            p, m, v = adam_update(p, m, v, g, t, lr)
    return p
