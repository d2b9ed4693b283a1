"""Pins of the damping-MLP oracle: finite differences, closed forms."""
import numpy as np

from oracle import mlp


def test_layout_and_init():
    nout = 4
    th = mlp.glorot_init(nout, 0)
    assert th.size == mlp.nparams(nout) == 64 * 3 + 64 + 64 * 64 + 64 + 4 * 64 + 4
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th, nout)
    assert np.all(b1 == 0) and np.all(b3 == 0)
    assert np.max(np.abs(W2)) <= np.sqrt(6 / 128) and np.max(np.abs(W1)) <= np.sqrt(6 / 67)


def test_forward_closed_form_zero_weights():
    nout = 3
    th = np.zeros(mlp.nparams(nout))
    y, _ = mlp.forward(th, np.random.default_rng(0).normal(size=(5, 3)), nout)
    assert np.allclose(y, 1.0)          # 2 sigmoid(0) = 1: the paper's omega


def test_backward_matches_finite_differences():
    nout = 4
    rng = np.random.default_rng(1)
    th = mlp.glorot_init(nout, 3) + 0.05 * rng.normal(size=mlp.nparams(nout))
    x = rng.uniform(0, 1, size=(7, 3))
    t = rng.uniform(0.5, 1.5, size=(7, nout))
    m = (rng.uniform(size=(7, nout)) < 0.7).astype(float)

    def L(theta):
        y, _ = mlp.forward(theta, x, nout)
        return mlp.loss(y, t, m)[0]

    y, cache = mlp.forward(th, x, nout)
    _, dy = mlp.loss(y, t, m)
    g = mlp.backward(th, cache, dy, nout)
    idx = rng.choice(th.size, size=60, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = 1e-6
        fd = (L(th + e) - L(th - e)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_is_lr_sign():
    th = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    th1, m, v = mlp.adam_step(th, g, np.zeros(5), np.zeros(5), 1, lr=0.01)
    # after bias correction the first step is lr * g / (|g| + eps)
    assert np.allclose(th1, -0.01 * g / (np.abs(g) + 1e-8))


def test_training_reduces_loss():
    nout = 2
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(32, 3))
    t = np.stack([1 + 0.4 * np.sin(3 * x[:, 0]), 0.8 + 0.3 * x[:, 1]], axis=1)
    m = np.ones_like(t)
    th = mlp.glorot_init(nout, 0)
    mm, vv = np.zeros_like(th), np.zeros_like(th)
    l0 = mlp.loss(mlp.forward(th, x, nout)[0], t, m)[0]
    for k in range(1, 301):
        y, c = mlp.forward(th, x, nout)
        _, dy = mlp.loss(y, t, m)
        th, mm, vv = mlp.adam_step(th, mlp.backward(th, c, dy, nout), mm, vv, k, lr=3e-3)
    l1 = mlp.loss(mlp.forward(th, x, nout)[0], t, m)[0]
    assert l1 < 0.1 * l0
