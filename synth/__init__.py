"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the solver method: only random arrays,
manufactured-solution parameters (the continuous functions u and
f = lambda u - Laplace u), and the mesh-width recipes that describe a
workload.  Both the HIP path and the oracle take their inputs from here.

Workload recipes (stand-ins for the paper's test problems, which use
inhomogeneous Dirichlet data on (0, 2 pi)^3):
* random right-hand sides, U(-1, 1) at every grid node (Sec. 5.2 uses
  pseudo-random input to avoid over-resolved data);
* sums of sine modes vanishing on the box boundary;
* geometrically stretched widths h_k ~ alpha^k (Sec. 5.4);
* anisotropic bricks on (0, AR) x (0, ceil(AR/2)/2) x (0, 1) (Sec. 5.3,
  scaled to unit height).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def random_grid(shape, seed):
    """U(-1, 1) values on a node grid of the given shape (float64)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)


def sine_modes(seed, n_modes=8, kmax=4):
    """Integer wave numbers k[m, d] in [1, kmax] and amplitudes a[m] ~ U(-1, 1)."""
    r = np.random.default_rng(seed)
    k = r.integers(1, kmax + 1, size=(n_modes, 3))
    a = r.uniform(-1.0, 1.0, size=n_modes)
    return k, a


def product_mode():
    """The single mode sin(pi x) sin(pi y) sin(pi z)."""
    return np.array([[1, 1, 1]]), np.array([1.0])


def sine_solution(k, a, lengths, x1, x2, x3, lam, xp=np):
    """Exact u and f = lam u - Laplace u for u = sum_m a_m prod_d sin(pi k_md x_d / l_d).

    x1, x2, x3 are broadcastable coordinate arrays (x1 varies fastest in
    the node grids); ``xp`` is numpy or torch.
    """
    u = 0.0
    f = 0.0
    for m in range(len(a)):
        s = (xp.sin(math.pi * float(k[m, 0]) * x1 / lengths[0])
             * xp.sin(math.pi * float(k[m, 1]) * x2 / lengths[1])
             * xp.sin(math.pi * float(k[m, 2]) * x3 / lengths[2]))
        kk = sum((math.pi * float(k[m, d]) / lengths[d]) ** 2 for d in range(3))
        u = u + float(a[m]) * s
        f = f + float(a[m]) * (lam + kk) * s
    return u, f


def paper_test_solution(k, lam, x1, x2, x3, xp=np):
    """Manufactured solution of the paper's runtime tests (Sec. 5.2) and its
    right-hand side f = lam u - Laplace u, on broadcastable coordinates
    (``xp`` is numpy or torch).

    u = cos(k(x1 - 3x2 + 2x3)) sin(k(1 + x1)) sin(k(1 - x2)) sin(k(2x1 + x2))
        sin(k(3x1 - 2x2 + 2x3)); the paper poses it on (0, 2 pi)^3 with k = 5,
    lam = 0 and its values as Dirichlet data on the whole boundary.  Writing
    each factor as two complex exponentials makes u a sum of 32 plane waves
    c_s exp(i (K_s.x + B_s)) over the sign choices s; the coefficients
    c_s = prod(sine signs) / 32 are real and s, -s give conjugate waves, so
    u = sum over 16 sign choices of 2 c_s cos(K_s.x + B_s), and Laplace u
    multiplies each term by -|K_s|^2.
    """
    # (wave vector / k, phase / k, cosine?) of the five factors
    factors = [((1.0, -3.0, 2.0), 0.0, True), ((1.0, 0.0, 0.0), 1.0, False),
               ((0.0, -1.0, 0.0), 1.0, False), ((2.0, 1.0, 0.0), 0.0, False),
               ((3.0, -2.0, 2.0), 0.0, False)]
    u = 0.0
    lap = 0.0
    for rest in itertools.product((1.0, -1.0), repeat=4):
        signs = (1.0,) + rest
        K = [0.0, 0.0, 0.0]
        B = 0.0
        c = 2.0 / 32.0
        for (a, b, is_cos), s in zip(factors, signs):
            K = [K[i] + s * k * a[i] for i in range(3)]
            B += s * k * b
            if not is_cos:
                c *= s
        wave = c * xp.cos(K[0] * x1 + K[1] * x2 + K[2] * x3 + B)
        u = u + wave
        lap = lap - (K[0] ** 2 + K[1] ** 2 + K[2] ** 2) * wave
    return u, lam * u - lap


def stretched_widths(n, alpha, length=1.0):
    h = alpha ** np.arange(n, dtype=np.float64)
    return h * (length / h.sum())


def anisotropic_widths(n, ar):
    """Uniform bricks on (0, AR) x (0, ceil(AR/2)/2) x (0, 1), n per direction."""
    lx, ly, lz = float(ar), math.ceil(ar / 2.0) / 2.0, 1.0
    return (np.full(n, lx / n), np.full(n, ly / n), np.full(n, lz / n)), (lx, ly, lz)
