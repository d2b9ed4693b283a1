"""Cartesian tensor-product meshes of cuboid elements (oracle).

Sec. 2.1: elements are cuboids of dimensions h_{1,e} x h_{2,e} x h_{3,e};
Sec. 5.4: geometrically stretched meshes with a constant expansion factor
alpha (h_{k+1} = alpha h_k, maximum aspect ratio alpha^(n-1));
Sec. 5.3: anisotropic brick meshes.  Homogeneous Dirichlet conditions on the
whole boundary.

Node grids have shape (N3, N2, N1), N_d = n_d p + 1, x1 fastest.  Element
e = (e1, e2, e3) owns the nodes i_d in [e_d p, e_d p + p].
"""
from __future__ import annotations

import numpy as np

from . import sem1d


def uniform_widths(n: int, length: float = 1.0):
    return np.full(n, length / n)


def stretched_widths(n: int, alpha: float, length: float = 1.0):
    """h_k proportional to alpha^k, k = 0..n-1, summing to ``length``."""
    h = alpha ** np.arange(n, dtype=np.float64)
    return h * (length / h.sum())


class Mesh:
    """Element widths per direction, polynomial degree and Helmholtz lambda."""

    def __init__(self, hx, hy, hz, p: int, lam: float):
        self.h = [np.asarray(hx, dtype=np.float64),
                  np.asarray(hy, dtype=np.float64),
                  np.asarray(hz, dtype=np.float64)]
        self.n = [len(h) for h in self.h]
        self.p = int(p)
        self.lam = float(lam)
        self.N = [nd * self.p + 1 for nd in self.n]
        self.shape = (self.N[2], self.N[1], self.N[0])

    @classmethod
    def box(cls, n, p, lam, alpha=1.0, lengths=(1.0, 1.0, 1.0)):
        if np.isscalar(n):
            n = (n, n, n)
        ws = [stretched_widths(n[d], alpha, lengths[d]) for d in range(3)]
        return cls(ws[0], ws[1], ws[2], p, lam)

    def with_degree(self, p: int) -> "Mesh":
        return Mesh(self.h[0], self.h[1], self.h[2], p, self.lam)

    # ---- coordinates --------------------------------------------------
    def coords_1d(self, d: int):
        x, _ = sem1d.gll(self.p)
        out = np.zeros(self.N[d])
        x0 = 0.0
        for e, h in enumerate(self.h[d]):
            out[e * self.p: e * self.p + self.p + 1] = x0 + h * (x + 1.0) / 2.0
            x0 += h
        out[-1] = x0
        return out

    def coords(self):
        """Broadcastable coordinate arrays (X3, X2, X1) of the node grid."""
        x1, x2, x3 = (self.coords_1d(d) for d in range(3))
        return x3[:, None, None], x2[None, :, None], x1[None, None, :]

    # ---- node classes -------------------------------------------------
    def dirichlet_mask(self):
        m = np.zeros(self.shape, dtype=bool)
        m[0, :, :] = m[-1, :, :] = True
        m[:, 0, :] = m[:, -1, :] = True
        m[:, :, 0] = m[:, :, -1] = True
        return m

    def skeleton_mask(self):
        """Element-boundary nodes (faces, edges, vertices), incl. Dirichlet."""
        p = self.p
        i3, i2, i1 = np.meshgrid(np.arange(self.N[2]), np.arange(self.N[1]),
                                 np.arange(self.N[0]), indexing="ij")
        return (i1 % p == 0) | (i2 % p == 0) | (i3 % p == 0)

    def free_skeleton_mask(self):
        """Unknowns of the condensed system: skeleton minus Dirichlet nodes."""
        return self.skeleton_mask() & ~self.dirichlet_mask()

    def interior_mask(self):
        return ~self.skeleton_mask()

    def n_elements(self):
        return self.n[0] * self.n[1] * self.n[2]

    def element_index_arrays(self):
        """Flat grid index of every local node of every element.

        Returns (idx, e1, e2, e3): idx has shape (n_e, p+1, p+1, p+1) with
        local order [i3, i2, i1]; e_d are the element coordinates (n_e,).
        """
        p = self.p
        n1, n2, n3 = self.n
        N1, N2, _ = self.N
        e3, e2, e1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1),
                                 indexing="ij")
        e1, e2, e3 = e1.ravel(), e2.ravel(), e3.ravel()
        loc = np.arange(p + 1)
        g3 = e3[:, None] * p + loc[None, :]
        g2 = e2[:, None] * p + loc[None, :]
        g1 = e1[:, None] * p + loc[None, :]
        idx = (g3[:, :, None, None] * N2 + g2[:, None, :, None]) * N1 \
            + g1[:, None, None, :]
        return idx, e1, e2, e3

    def assembled_mass(self):
        """Diagonal of the assembled GLL mass matrix on the node grid."""
        m = [np.zeros(self.N[d]) for d in range(3)]
        for d in range(3):
            for e, h in enumerate(self.h[d]):
                me, _ = sem1d.element_matrices(self.p, h)
                m[d][e * self.p: e * self.p + self.p + 1] += me
        return m[2][:, None, None] * m[1][None, :, None] * m[0][None, None, :]

    def n_dof(self):
        """Unknown count n_e * p^3 used as the throughput convention."""
        return self.n_elements() * self.p ** 3


def level_degrees(p: int, p0: int = 2):
    """p-multigrid degrees (Sec. 4.1): p_l = p0 2^l for l < L, p_L = p.

    L is the smallest integer with p0 2^L >= p, so the top level carries p
    itself and the level below it is the largest power-of-two multiple of p0
    that is smaller than p.
    """
    if p <= p0:
        return [p]
    degs = [p0]
    while degs[-1] * 2 < p:
        degs.append(degs[-1] * 2)
    degs.append(p)
    return degs
