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


def test_adam_constant_gradient_steps():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each
    step moves by lr g / (|g| + eps): theta_t = theta_0 - t lr g / (|g| + eps).
    A wrong exponent in either bias correction breaks this for t > 1."""
    g = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    th, m, v = np.zeros(5), np.zeros(5), np.zeros(5)
    for t in range(1, 8):
        th, m, v = mlp.adam_step(th, g, m, v, t, lr=0.01, b1=0.8, b2=0.9)
        assert np.allclose(m, (1 - 0.8 ** t) * g, rtol=1e-14, atol=0)
        assert np.allclose(v, (1 - 0.9 ** t) * g * g, rtol=1e-14, atol=0)
        assert np.allclose(th, -t * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_moments_closed_form():
    """Alternating gradients +g, -g: m_t = (1 - b1) sum_k b1^(t-k) g_k and
    v_t = (1 - b2^t) g^2 in closed form; the step uses m_t / (1 - b1^t)
    over sqrt(v_t / (1 - b2^t)) + eps."""
    g0 = np.array([0.3, -1.5])
    b1, b2, lr, eps = 0.9, 0.99, 0.1, 1e-8
    th, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    th_ref = np.zeros(2)
    for t in range(1, 6):
        gt = g0 * (-1) ** (t + 1)
        th, m, v = mlp.adam_step(th, gt, m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        mt = (1 - b1) * sum(b1 ** (t - k) * g0 * (-1) ** (k + 1) for k in range(1, t + 1))
        vt = (1 - b2 ** t) * g0 * g0
        th_ref = th_ref - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        assert np.allclose(m, mt, rtol=1e-13) and np.allclose(v, vt, rtol=1e-13)
        assert np.allclose(th, th_ref, rtol=1e-12)


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
