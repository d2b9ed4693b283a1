"""Damping-weight MLP 3 -> 64 -> 64 -> L (oracle, FP64).

Not part of the paper: the per-level damping omega_l of the smoother
(u_l += omega_l Smoother(r_l); omega_l = 1 is the paper's method) is
predicted by a small network from (p, lambda h^2, aspect ratio).

Network:  h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2),
          y = 2 sigmoid(W3 h2 + b3)         (y in (0, 2))
Loss:     masked mean squared error, sum m (y - t)^2 / sum m
Update:   Adam (Kingma & Ba 2015) with bias correction.
Parameter vector layout: W1[64][3], b1[64], W2[64][64], b2[64],
W3[L][64], b3[L] (row-major), identical to the C ABI.
"""
from __future__ import annotations

import numpy as np

H = 64


def nparams(nout):
    return H * 3 + H + H * H + H + nout * H + nout


def unpack(theta, nout):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    out = []
    for shape in ((H, 3), (H,), (H, H), (H,), (nout, H), (nout,)):
        n = int(np.prod(shape))
        out.append(theta[o:o + n].reshape(shape))
        o += n
    return out


def glorot_init(nout, seed):
    """Glorot-uniform weights, zero biases."""
    r = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((3, H), (H, H), (H, nout)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(r.uniform(-lim, lim, size=(fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def forward(theta, x, nout):
    W1, b1, W2, b2, W3, b3 = unpack(theta, nout)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    s = h2 @ W3.T + b3
    y = 2.0 / (1.0 + np.exp(-s))
    return y, (x, h1, h2, y)


def loss(y, t, m):
    cnt = max(float(np.sum(m)), 1.0)
    return float(np.sum(m * (y - t) ** 2) / cnt), 2.0 * m * (y - t) / cnt


def backward(theta, cache, dy, nout):
    """Gradient of sum_b dy_b . y_b with respect to theta (analytic)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, nout)
    x, h1, h2, y = cache
    ds = dy * y * (1.0 - 0.5 * y)          # d(2 sigma(s))/ds = y (1 - y/2)
    gW3 = ds.T @ h2
    gb3 = ds.sum(axis=0)
    dh2 = (ds @ W3) * (1.0 - h2 ** 2)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (1.0 - h1 ** 2)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
