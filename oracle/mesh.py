"""Cartesian tensor-product meshes of cuboid elements (oracle).

Sec. 2.1: elements are cuboids of dimensions h_{1,e} x h_{2,e} x h_{3,e};
Sec. 5.4: geometrically stretched meshes with a constant expansion factor
alpha (h_{k+1} = alpha h_k, maximum aspect ratio alpha^(n-1));
Sec. 5.3: anisotropic brick meshes.

Boundary conditions (Sec. 3.3) are set per direction and side: homogeneous
Dirichlet ("D", the default on every side), homogeneous Neumann ("N": the
boundary nodes are unknowns and the natural condition holds), or periodic
("P", both sides of a direction).  In a periodic direction the last node
layer i_d = N_d - 1 is the first one again: the grid keeps it as a mirror
entry that holds no unknown, and the element-to-node map wraps onto the
first layer, so the two neighbours of the seam are coupled by assembly.

Node grids have shape (N3, N2, N1), N_d = n_d p + 1, x1 fastest.  Element
e = (e1, e2, e3) owns the nodes i_d in [e_d p, e_d p + p] (taken modulo
N_d - 1 in a periodic direction).
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


def parse_bc(bc):
    """Normalise a boundary specification to ((lo, hi), ...) per direction.

    ``bc`` is None (Dirichlet everywhere) or three entries, each "P"
    (periodic), a single kind "D"/"N" for both sides, or a pair (lo, hi) of
    kinds; a six-letter string "DNPPDD" lists (lo, hi) for x1, x2, x3.
    """
    if bc is None:
        return (("D", "D"),) * 3
    if isinstance(bc, str) and len(bc) == 6:
        bc = [bc[0:2], bc[2:4], bc[4:6]]
    out = []
    for b in bc:
        if isinstance(b, str) and len(b) == 1:
            b = (b, b)
        lo, hi = b[0], b[1]
        if lo not in "DNP" or hi not in "DNP" or (("P" in (lo, hi)) and lo != hi):
            raise ValueError(f"bad boundary specification {bc!r}")
        out.append((lo, hi))
    return tuple(out)


class Mesh:
    """Element widths per direction, polynomial degree, Helmholtz lambda and
    boundary conditions."""

    def __init__(self, hx, hy, hz, p: int, lam: float, bc=None):
        self.h = [np.asarray(hx, dtype=np.float64),
                  np.asarray(hy, dtype=np.float64),
                  np.asarray(hz, dtype=np.float64)]
        self.n = [len(h) for h in self.h]
        self.p = int(p)
        self.lam = float(lam)
        self.N = [nd * self.p + 1 for nd in self.n]
        self.shape = (self.N[2], self.N[1], self.N[0])
        self.bc = parse_bc(bc)
        self.periodic = [self.bc[d][0] == "P" for d in range(3)]
        if not any("D" in b for b in self.bc) and self.lam <= 0.0:
            raise ValueError("without a Dirichlet side the operator is singular for lambda <= 0")
        for d in range(3):
            if self.periodic[d] and self.n[d] < 3:
                raise ValueError("a periodic direction needs at least 3 elements")

    @classmethod
    def box(cls, n, p, lam, alpha=1.0, lengths=(1.0, 1.0, 1.0), bc=None):
        if np.isscalar(n):
            n = (n, n, n)
        ws = [stretched_widths(n[d], alpha, lengths[d]) for d in range(3)]
        return cls(ws[0], ws[1], ws[2], p, lam, bc)

    def with_degree(self, p: int) -> "Mesh":
        return Mesh(self.h[0], self.h[1], self.h[2], p, self.lam, self.bc)

    def all_dirichlet(self) -> bool:
        return all(b == ("D", "D") for b in self.bc)

    # ---- index maps -----------------------------------------------------
    def global_1d(self, d: int):
        """(n_d, p+1) node index of local node a of element e in direction d:
        e p + a, wrapped modulo N_d - 1 in a periodic direction."""
        g = np.arange(self.n[d])[:, None] * self.p + np.arange(self.p + 1)[None, :]
        if self.periodic[d]:
            g = g % (self.N[d] - 1)
        return g

    def wrap(self, d: int, i):
        """Node index i (possibly outside 0..N_d-1) taken onto the node grid:
        modulo N_d - 1 in a periodic direction, unchanged otherwise."""
        return np.mod(i, self.N[d] - 1) if self.periodic[d] else i

    def expand_periodic(self, grid):
        """Copy of a node grid with each periodic direction's last layer set
        to its first (the mirror entries repeat the unknowns they stand for)."""
        g = np.array(grid, dtype=np.float64, copy=True)
        if self.periodic[0]:
            g[:, :, -1] = g[:, :, 0]
        if self.periodic[1]:
            g[:, -1, :] = g[:, 0, :]
        if self.periodic[2]:
            g[-1, :, :] = g[0, :, :]
        return g

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
        (a1, b1), (a2, b2), (a3, b3) = self.bc
        if a3 == "D":
            m[0, :, :] = True
        if b3 == "D":
            m[-1, :, :] = True
        if a2 == "D":
            m[:, 0, :] = True
        if b2 == "D":
            m[:, -1, :] = True
        if a1 == "D":
            m[:, :, 0] = True
        if b1 == "D":
            m[:, :, -1] = True
        return m

    def mirror_mask(self):
        """Last node layer of each periodic direction (no unknown of its own)."""
        m = np.zeros(self.shape, dtype=bool)
        if self.periodic[0]:
            m[:, :, -1] = True
        if self.periodic[1]:
            m[:, -1, :] = True
        if self.periodic[2]:
            m[-1, :, :] = True
        return m

    def skeleton_mask(self):
        """Element-boundary nodes (faces, edges, vertices), incl. Dirichlet."""
        p = self.p
        i3, i2, i1 = np.meshgrid(np.arange(self.N[2]), np.arange(self.N[1]),
                                 np.arange(self.N[0]), indexing="ij")
        return (i1 % p == 0) | (i2 % p == 0) | (i3 % p == 0)

    def free_skeleton_mask(self):
        """Unknowns of the condensed system: skeleton minus Dirichlet and
        mirror nodes."""
        return self.skeleton_mask() & ~self.dirichlet_mask() & ~self.mirror_mask()

    def free_mask(self):
        """All unknowns of the full system (interior included)."""
        return ~self.dirichlet_mask() & ~self.mirror_mask()

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
        g3 = self.global_1d(2)[e3]
        g2 = self.global_1d(1)[e2]
        g1 = self.global_1d(0)[e1]
        idx = (g3[:, :, None, None] * N2 + g2[:, None, :, None]) * N1 \
            + g1[:, None, None, :]
        return idx, e1, e2, e3

    def assembled_mass(self):
        """Diagonal of the assembled GLL mass matrix on the node grid."""
        m = [np.zeros(self.N[d]) for d in range(3)]
        for d in range(3):
            g = self.global_1d(d)
            for e, h in enumerate(self.h[d]):
                me, _ = sem1d.element_matrices(self.p, h)
                np.add.at(m[d], g[e], me)
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
