"""Dense plain-definition routes on tiny meshes (oracle, FP64).

Everything here assembles matrices explicitly and uses dense linear algebra,
so it is only usable for a few hundred to a few thousand unknowns.  It pins
the matrix-free routes in ``matfree``:

* global operator  H = sum_e Q_e H_e Q_e^T          (Sec. 2.1)
* condensed system Hhat = H_BB - H_BI H_II^-1 H_IB,
                   Fhat = F_B - H_BI H_II^-1 F_I     (Sec. 2.2)
* star operator    Hhat_i = R_i Hhat R_i^T           (Sec. 2.3)
* smoother         sum_i W_i R_i^T Hhat_i^-1 R_i     (eq. smoother_definition)
* prolongation     tensor-product Lagrange interpolation restricted to the
                   condensed unknowns, restriction = its transpose (Sec. 4.1)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import sem1d
from .mesh import Mesh


def element_operator(p, h1, h2, h3, lam):
    """H_e = lam M3xM2xM1 + M3xM2xL1 + M3xL2xM1 + L3xM2xM1, order [i3,i2,i1].

    This is eq. (helmholtzop) with the d_e coefficients folded into the
    physical 1D matrices (h/2) M and (2/h) L.
    """
    m1, L1 = sem1d.element_matrices(p, h1)
    m2, L2 = sem1d.element_matrices(p, h2)
    m3, L3 = sem1d.element_matrices(p, h3)
    M1, M2, M3 = np.diag(m1), np.diag(m2), np.diag(m3)
    k = np.kron
    return (lam * k(M3, k(M2, M1)) + k(M3, k(M2, L1)) + k(M3, k(L2, M1))
            + k(L3, k(M2, M1)))


def assemble_H(mesh: Mesh):
    """Dense global operator over all grid nodes (Dirichlet rows kept)."""
    idx, e1, e2, e3 = mesh.element_index_arrays()
    ntot = int(np.prod(mesh.shape))
    H = np.zeros((ntot, ntot))
    p = mesh.p
    for e in range(len(e1)):
        He = element_operator(p, mesh.h[0][e1[e]], mesh.h[1][e2[e]],
                              mesh.h[2][e3[e]], mesh.lam)
        g = idx[e].ravel()
        H[np.ix_(g, g)] += He
    return H


class CondensedSystem:
    """Dense Schur complement of H onto the free skeleton unknowns."""

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        self.H = assemble_H(mesh)
        self.B = np.flatnonzero(mesh.free_skeleton_mask().ravel())
        self.I = np.flatnonzero(mesh.interior_mask().ravel())
        H = self.H
        self.HBB = H[np.ix_(self.B, self.B)]
        self.HBI = H[np.ix_(self.B, self.I)]
        self.HIB = H[np.ix_(self.I, self.B)]
        self.HII = H[np.ix_(self.I, self.I)]
        if len(self.I):
            self.HII_inv_HIB = np.linalg.solve(self.HII, self.HIB)
            self.Hhat = self.HBB - self.HBI @ self.HII_inv_HIB
        else:
            self.Hhat = self.HBB.copy()
        self.pos = {g: k for k, g in enumerate(self.B)}

    def to_vec(self, grid):
        return np.asarray(grid).ravel()[self.B]

    def to_grid(self, vec):
        g = np.zeros(int(np.prod(self.mesh.shape)))
        g[self.B] = vec
        return g.reshape(self.mesh.shape)

    def condense_rhs(self, F_grid):
        F = np.asarray(F_grid).ravel()
        FB, FI = F[self.B], F[self.I]
        if len(self.I):
            return FB - self.HBI @ np.linalg.solve(self.HII, FI)
        return FB

    def recover(self, F_grid, uhat):
        """Full nodal solution from the skeleton solution (Alg. 4, last step)."""
        F = np.asarray(F_grid).ravel()
        u = np.zeros(F.size)
        u[self.B] = uhat
        if len(self.I):
            u[self.I] = np.linalg.solve(self.HII, F[self.I] - self.HIB @ uhat)
        return u.reshape(self.mesh.shape)

    def full_solve(self, F_grid):
        """u* = H^-1 F on the unknowns (brute force); mirror entries of a
        periodic direction repeat the first layer."""
        free = np.flatnonzero(self.mesh.free_mask().ravel())
        F = np.asarray(F_grid).ravel()
        u = np.zeros(F.size)
        u[free] = np.linalg.solve(self.H[np.ix_(free, free)], F[free])
        return self.mesh.expand_periodic(u.reshape(self.mesh.shape))

    # ---- stars ---------------------------------------------------------
    def star_nodes(self, v):
        """Free skeleton nodes of the star around vertex v = (v1, v2, v3).

        The star consists of the three planes through the vertex, restricted
        to the window of offsets -(p-1)..(p-1) in every direction; in a
        periodic direction the window continues across the seam.
        Returns (flat grid indices, offsets (k, 3) as (o1, o2, o3)).
        """
        m = self.mesh
        p = m.p
        ctr = [v[d] * p for d in range(3)]
        out, offs = [], []
        rng = range(-(p - 1), p)
        for o3 in rng:
            for o2 in rng:
                for o1 in rng:
                    if o1 != 0 and o2 != 0 and o3 != 0:
                        continue
                    i1, i2, i3 = ctr[0] + o1, ctr[1] + o2, ctr[2] + o3
                    i1, i2, i3 = (int(m.wrap(0, i1)), int(m.wrap(1, i2)),
                                  int(m.wrap(2, i3)))
                    if not (0 <= i1 < m.N[0] and 0 <= i2 < m.N[1]
                            and 0 <= i3 < m.N[2]):
                        continue
                    g = (i3 * m.N[1] + i2) * m.N[0] + i1
                    if g in self.pos:
                        out.append(g)
                        offs.append((o1, o2, o3))
        return np.array(out, dtype=np.int64), np.array(offs).reshape(-1, 3)

    def vertices(self):
        m = self.mesh
        n1, n2, n3 = (m.n[d] + (0 if m.periodic[d] else 1) for d in range(3))
        return [(a, b, c) for c in range(n3) for b in range(n2)
                for a in range(n1)]

    def star_operator(self, v):
        g, _ = self.star_nodes(v)
        k = np.array([self.pos[x] for x in g], dtype=np.int64)
        return self.Hhat[np.ix_(k, k)], k

    def smoother_matrix(self, omega=1.0, pw=7, unit_weights=False):
        """Dense sum_i W_i R_i^T Hhat_i^-1 R_i over all vertices (Alg. 2)."""
        p = self.mesh.p
        w1 = sem1d.star_weights_1d(p, pw)
        nB = len(self.B)
        Smat = np.zeros((nB, nB))
        for v in self.vertices():
            g, offs = self.star_nodes(v)
            if len(g) == 0:
                continue
            k = np.array([self.pos[x] for x in g], dtype=np.int64)
            Hi = self.Hhat[np.ix_(k, k)]
            Hi_inv = scipy.linalg.inv(Hi)
            if unit_weights:
                W = np.ones(len(k))
            else:
                W = (w1[offs[:, 0] + p - 1] * w1[offs[:, 1] + p - 1]
                     * w1[offs[:, 2] + p - 1])
            Smat[np.ix_(k, k)] += W[:, None] * Hi_inv
        return omega * Smat


def block_nodes(cs: CondensedSystem, e):
    """Free skeleton nodes of the element-centred block of element e.

    The block covers the open region ((e_d - 1) p, (e_d + 2) p) in every
    direction (3 x 3 x 3 elements around e, Sec. 3.4); its condensed
    unknowns are all free skeleton nodes inside.  Returns (flat grid
    indices, positions (k, 3) as (o1, o2, o3) with o_d = i_d - (e_d - 1) p - 1).
    """
    m = cs.mesh
    p = m.p
    lo = [(e[d] - 1) * p for d in range(3)]
    rng = []
    for d in range(3):          # positions along d: the open block, across a periodic seam
        if m.periodic[d]:
            rng.append(range(lo[d] + 1, lo[d] + 3 * p))
        else:
            rng.append(range(max(lo[d] + 1, 0), min(lo[d] + 3 * p, m.N[d])))
    out, offs = [], []
    for i3 in rng[2]:
        for i2 in rng[1]:
            for i1 in rng[0]:
                j1, j2, j3 = int(m.wrap(0, i1)), int(m.wrap(1, i2)), int(m.wrap(2, i3))
                g = (j3 * m.N[1] + j2) * m.N[0] + j1
                if g in cs.pos:
                    out.append(g)
                    offs.append((i1 - lo[0] - 1, i2 - lo[1] - 1, i3 - lo[2] - 1))
    return np.array(out, dtype=np.int64), np.array(offs).reshape(-1, 3)


def block_smoother_matrix(cs: CondensedSystem, omega=1.0, weights="smooth", unit_weights=False):
    """Dense sum_e W_e R_e^T Hhat_e^-1 R_e over all element-centred blocks,
    with Hhat_e = R_e Hhat R_e^T inverted by dense LU."""
    from .blocks import block_weights_1d
    m = cs.mesh
    p = m.p
    nB = len(cs.B)
    Smat = np.zeros((nB, nB))
    for e3 in range(m.n[2]):
        for e2 in range(m.n[1]):
            for e1 in range(m.n[0]):
                e = (e1, e2, e3)
                g, offs = block_nodes(cs, e)
                if len(g) == 0:
                    continue
                k = np.array([cs.pos[x] for x in g], dtype=np.int64)
                Hi_inv = scipy.linalg.inv(cs.Hhat[np.ix_(k, k)])
                if unit_weights:
                    W = np.ones(len(k))
                else:
                    w = [block_weights_1d(m.n[d], p, e[d], weights, periodic=m.periodic[d]) for d in range(3)]
                    W = w[0][offs[:, 0]] * w[1][offs[:, 1]] * w[2][offs[:, 2]]
                Smat[np.ix_(k, k)] += W[:, None] * Hi_inv
    return omega * Smat


def interp_1d_global(hs, pc, pf):
    """Global 1D interpolation from degree pc to pf on elements ``hs``.

    Rows: fine nodes (n pf + 1); columns: coarse nodes (n pc + 1).  The
    element-local block is the Lagrange matrix between the GLL nodes of the
    two degrees; element-boundary rows are unit rows shared by neighbours.
    """
    n = len(hs)
    xc, _ = sem1d.gll(pc)
    xf, _ = sem1d.gll(pf)
    J = sem1d.lagrange_matrix(xc, xf)
    P = np.zeros((n * pf + 1, n * pc + 1))
    for e in range(n):
        P[e * pf: e * pf + pf + 1, e * pc: e * pc + pc + 1] = J
    return P


def prolongation_matrix(mesh_c: Mesh, mesh_f: Mesh):
    """Dense P: coarse free skeleton -> fine free skeleton (Sec. 4.1)."""
    P1 = interp_1d_global(mesh_c.h[0], mesh_c.p, mesh_f.p)
    P2 = interp_1d_global(mesh_c.h[1], mesh_c.p, mesh_f.p)
    P3 = interp_1d_global(mesh_c.h[2], mesh_c.p, mesh_f.p)
    full = np.kron(P3, np.kron(P2, P1))
    # periodic: the value at a coarse mirror node is the value at the node
    # it repeats, so its column adds to that node's column
    Nc = mesh_c.N
    i3, i2, i1 = np.meshgrid(np.arange(Nc[2]), np.arange(Nc[1]), np.arange(Nc[0]), indexing="ij")
    j1, j2, j3 = mesh_c.wrap(0, i1), mesh_c.wrap(1, i2), mesh_c.wrap(2, i3)
    canon = ((j3 * Nc[1] + j2) * Nc[0] + j1).ravel()
    folded = np.zeros_like(full)
    for col in range(full.shape[1]):
        folded[:, canon[col]] += full[:, col]
    rows = np.flatnonzero(mesh_f.free_skeleton_mask().ravel())
    cols = np.flatnonzero(mesh_c.free_skeleton_mask().ravel())
    return folded[np.ix_(rows, cols)]
