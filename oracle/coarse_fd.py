"""Exact coarse solve by fast diagonalization (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU baseline use this package; the product path never does.

On a Cartesian mesh the assembled operator of any degree is the tensor sum
H = lam M3 x M2 x M1 + M3 x M2 x L1 + M3 x L2 x M1 + L3 x M2 x M1 of the
assembled 1D GLL mass (diagonal) and stiffness matrices (Sec. 2.1, eq.
helmholtzop), Dirichlet nodes removed (a Neumann end node stays, a periodic
direction is assembled on its n p distinct nodes).  With the generalized eigenpairs
S_d^T L_d S_d = diag(mu_d), S_d^T M_d S_d = I, its inverse is
(S3 x S2 x S1) diag(1 / (lam + mu1 + mu2 + mu3)) (S3 x S2 x S1)^T (eq.
fast_diagonalization, here on the whole mesh instead of a star).

The condensed system Hhat u_B = F_B (Sec. 2.2) is the skeleton part of the
full system H [u_B; u_I] = [F_B; 0]: the second block row gives
u_I = -H_II^-1 H_IB u_B, and substituting it into the first leaves
(H_BB - H_BI H_II^-1 H_IB) u_B = F_B.  So the exact coarse solve of the
condensed p-multigrid hierarchy is one fast-diagonalization solve of the
full coarse system with zero right-hand side in the element interiors.
The paper solves the coarse problem by CG (Sec. 4.1) and does not fix a
tolerance; this exact solve is a reading that uses its own diagonalization.
"""
from __future__ import annotations

import numpy as np

from . import sem1d
from .mesh import Mesh


def assembled_1d(hs, p, periodic=False):
    """Assembled 1D mass (vector) and stiffness on the n p + 1 nodes of one
    direction with element widths hs; periodic: on the n p distinct nodes,
    the last element's end node being node 0."""
    n = len(hs)
    N = n * p if periodic else n * p + 1
    M = np.zeros(N)
    L = np.zeros((N, N))
    for e, h in enumerate(hs):
        m, Le = sem1d.element_matrices(p, h)
        g = (e * p + np.arange(p + 1)) % N
        np.add.at(M, g, m)
        L[np.ix_(g, g)] += Le
    return M, L


def unknown_range(mesh: Mesh, d: int):
    """Node indices of direction d that carry unknowns: Dirichlet ends
    dropped, the mirror end of a periodic direction dropped."""
    lo, hi = mesh.bc[d]
    a = 1 if lo == "D" else 0
    b = mesh.N[d] - (1 if hi in "DP" else 0)
    return a, b


def fd_tables(mesh: Mesh):
    """Per direction (S_d, mu_d) of the assembled 1D problem on the nodes
    that carry unknowns."""
    out = []
    for d in range(3):
        M, L = assembled_1d(mesh.h[d], mesh.p, mesh.periodic[d])
        a, b = unknown_range(mesh, d)
        if not mesh.periodic[d]:
            M, L = M[a:b], L[a:b, a:b]
        S, mu = sem1d.gen_eig(L, np.diag(M))
        out.append((S, mu))
    return out


def fd_solve_full(mesh: Mesh, F_grid):
    """u = H^-1 F on the unknowns (zero at Dirichlet nodes; mirror entries
    of a periodic direction repeat the first layer)."""
    (S1, m1), (S2, m2), (S3, m3) = fd_tables(mesh)
    r = [unknown_range(mesh, d) for d in range(3)]
    sl = (slice(*r[2]), slice(*r[1]), slice(*r[0]))
    X = np.asarray(F_grid, dtype=np.float64)[sl]     # [i3, i2, i1]
    X = np.einsum("ai,kji->kja", S1.T, X)
    X = np.einsum("bj,kjc->kbc", S2.T, X)
    X = np.einsum("ck,kji->cji", S3.T, X)
    X = X / (mesh.lam + m3[:, None, None] + m2[None, :, None] + m1[None, None, :])
    X = np.einsum("ia,kja->kji", S1, X)
    X = np.einsum("jb,kbc->kjc", S2, X)
    X = np.einsum("kc,cji->kji", S3, X)
    u = np.zeros(mesh.shape)
    u[sl] = X
    return mesh.expand_periodic(u)


def fd_condensed_solve(mesh: Mesh, F_grid):
    """u_B = Hhat^-1 F_B: the skeleton part of the full solve with the right-
    hand side kept on the free skeleton nodes and zero in the interiors."""
    mask = mesh.free_skeleton_mask()
    u = fd_solve_full(mesh, np.where(mask, F_grid, 0.0))
    return np.where(mask, u, 0.0)
