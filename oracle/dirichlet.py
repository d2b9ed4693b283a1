"""Inhomogeneous Dirichlet data by lifting (oracle, FP64).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The paper's runtime test problem (Sec. 5.2, the manufactured solution on
(0, 2 pi)^3) prescribes inhomogeneous Dirichlet values on the whole
boundary, and its boundary treatment (Sec. 3.3) keeps Dirichlet values
fixed while every correction vanishes there.  The discrete problem is:
u = g on the boundary nodes D, and on the free nodes f the rows of
H u = M f hold, i.e.

    H_ff u_f = (M f)_f - H_fD g_D.

With G = g on D and 0 elsewhere, u = u0 + G, where u0 vanishes on D and
solves the homogeneous problem with the right-hand side M f - H G on the
free nodes.  M is diagonal and positive, so that right-hand side is M f'
with f' = f - M^-1 H G, and the homogeneous solver applies unchanged to f'.

``exact_solve`` is the first display, written out with the dense assembled
operator; ``lift_rhs`` and ``solve`` are the lifting route.
"""
from __future__ import annotations

import numpy as np

from . import dense, matfree, solver
from .mesh import Mesh


def apply_H(mesh: Mesh, u_grid):
    """H u = sum_e Q_e H_e Q_e^T u over every grid node, boundary rows and
    columns kept (Sec. 2.1, eq. helmholtzop)."""
    el = matfree._elements(mesh)
    return el.scatter(el.He(el.gather(u_grid)))


def lift_rhs(mesh: Mesh, f_grid, g_grid):
    """f' = f - M^-1 H G on the free nodes and 0 on the boundary, where G
    takes the boundary values of g and is zero inside."""
    if not mesh.all_dirichlet():
        raise NotImplementedError("lifting: Dirichlet data on every side")
    D = mesh.dirichlet_mask()
    G = np.where(D, np.asarray(g_grid, dtype=np.float64), 0.0)
    fp = np.asarray(f_grid, dtype=np.float64) - apply_H(mesh, G) / mesh.assembled_mass()
    return np.where(D, 0.0, fp)


def solve(mesh: Mesh, f_grid, g_grid, method="kMG", rtol=1e-10, maxit=200, **hkw):
    """Solve with u = g on the boundary: lift, the homogeneous solve
    (Alg. 4 / Alg. 5), then the boundary values of g."""
    res = solver.solve(mesh, lift_rhs(mesh, f_grid, g_grid), method, rtol, maxit, **hkw)
    res.u = np.where(mesh.dirichlet_mask(), np.asarray(g_grid, dtype=np.float64), res.u)
    return res


def exact_solve(mesh: Mesh, f_grid, g_grid):
    if not mesh.all_dirichlet():
        raise NotImplementedError("lifting: Dirichlet data on every side")
    """Brute force on tiny meshes: u_D = g_D and
    u_f = H_ff^-1 ((M f)_f - H_fD g_D) with the dense assembled H."""
    H = dense.assemble_H(mesh)
    D = mesh.dirichlet_mask().ravel()
    fr = ~D
    F = (mesh.assembled_mass() * np.asarray(f_grid, dtype=np.float64)).ravel()
    g = np.asarray(g_grid, dtype=np.float64).ravel()
    u = np.where(D, g, 0.0)
    u[fr] = np.linalg.solve(H[np.ix_(fr, fr)], F[fr] - H[np.ix_(fr, D)] @ g[D])
    return u.reshape(mesh.shape)
