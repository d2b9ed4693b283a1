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


def paper_test_solution(k, lam, x1, x2, x3):
    """Manufactured solution of the paper's runtime tests (Sec. 5.2) and its
    right-hand side f = lam u - Laplace u, on broadcastable coordinates.

    u = cos(k(x1 - 3x2 + 2x3)) sin(k(1 + x1)) sin(k(1 - x2)) sin(k(2x1 + x2))
        sin(k(3x1 - 2x2 + 2x3)); the paper poses it on (0, 2 pi)^3 with k = 5,
    lam = 0 and its values as Dirichlet data on the whole boundary.  Each
    factor is written as two complex exponentials, so u is a sum of 32
    plane waves exp(i (K.x + B)) and Laplace u multiplies each by -|K|^2.
    """
    # (wave vector / k, phase / k, cosine?) of the five factors
    factors = [((1.0, -3.0, 2.0), 0.0, True), ((1.0, 0.0, 0.0), 1.0, False),
               ((0.0, -1.0, 0.0), 1.0, False), ((2.0, 1.0, 0.0), 0.0, False),
               ((3.0, -2.0, 2.0), 0.0, False)]
    u = 0.0
    lap = 0.0
    for signs in itertools.product((1.0, -1.0), repeat=5):
        K = np.zeros(3)
        B = 0.0
        c = 1.0 + 0.0j
        for (a, b, is_cos), s in zip(factors, signs):
            K = K + s * k * np.asarray(a)
            B += s * k * b
            c *= 0.5 if is_cos else s / 2.0j
        wave = c * np.exp(1j * (K[0] * x1 + K[1] * x2 + K[2] * x3 + B))
        u = u + wave
        lap = lap - float(K @ K) * wave
    u, lap = np.real(u), np.real(lap)
    return u, lam * u - lap


def stretched_widths(n, alpha, length=1.0):
    h = alpha ** np.arange(n, dtype=np.float64)
    return h * (length / h.sum())


def anisotropic_widths(n, ar):
    """Uniform bricks on (0, AR) x (0, ceil(AR/2)/2) x (0, 1), n per direction."""
    lx, ly, lz = float(ar), math.ceil(ar / 2.0) / 2.0, 1.0
    return (np.full(n, lx / n), np.full(n, ly / n), np.full(n, lz / n)), (lx, ly, lz)


def mlp_features(p, lam, hmin, ar):
    """Scaled inputs of the damping MLP: (p/32, log10(1+lam h^2)/4, log2(AR)/4)."""
    return np.array([p / 32.0, math.log10(1.0 + lam * hmin * hmin) / 4.0,
                     math.log2(max(ar, 1.0)) / 4.0], dtype=np.float32)
