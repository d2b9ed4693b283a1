"""Pins of the oracle's exact coarse solve by fast diagonalization: the
dense Schur-complement solve Hhat^-1 F_B and the dense full solve H^-1 F
(brute force on tiny meshes, degrees 1-3, stretched widths, lambda = 0), the
1D eigen identities of the assembled tables, and the V-cycle built on it
against the one with the dense exact coarse solve."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import coarse_fd, solver
from oracle import mesh as omesh
from oracle.dense import CondensedSystem

MESHES = [((3, 3, 3), 1, 1.0, 1.3), ((4, 3, 2), 2, 0.0, 1.0), ((2, 3, 2), 3, 2.0, 1.2),
          ((1, 2, 1), 2, 0.5, 1.0)]


@pytest.mark.parametrize("case", MESHES)
def test_fd_equals_dense_solves(case):
    n, p, lam, alpha = case
    m = omesh.Mesh.box(n, p, lam, alpha)
    cs = CondensedSystem(m)
    F = synth.random_grid(m.shape, 2) * m.free_skeleton_mask()
    ref = cs.to_grid(np.linalg.solve(cs.Hhat, cs.to_vec(F)))
    got = coarse_fd.fd_condensed_solve(m, F)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    Ff = synth.random_grid(m.shape, 3)
    full = cs.full_solve(Ff)
    assert np.linalg.norm(coarse_fd.fd_solve_full(m, Ff) - full) <= 1e-13 * np.linalg.norm(full)


def test_fd_tables_eigen_identities():
    m = omesh.Mesh.box((5, 3, 4), 2, 1.0, 1.4)
    for d, (S, mu) in enumerate(coarse_fd.fd_tables(m)):
        M, L = coarse_fd.assembled_1d(m.h[d], m.p)
        Mi, Li = np.diag(M[1:-1]), L[1:-1, 1:-1]
        assert S.shape == (m.N[d] - 2, m.N[d] - 2)
        assert np.allclose(S.T @ Mi @ S, np.eye(len(mu)), atol=1e-13)
        assert np.allclose(S.T @ Li @ S, np.diag(mu), atol=1e-11 * mu.max())


def test_vcycle_with_fd_coarse_equals_dense_coarse():
    m = omesh.Mesh.box((3, 2, 3), 8, 1.0, 1.2)
    r = synth.random_grid(m.shape, 4) * m.free_skeleton_mask()
    a = solver.Hierarchy(m, coarse="fd").vcycle(None, r)
    b = solver.Hierarchy(m, exact_coarse=True).vcycle(None, r)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_coarse_level_above_zero():
    """Exact coarse solve on p-level k > 0 (the levels below it dropped):
    with k = L the V-cycle is the exact condensed solve (dense
    Schur-complement solve); with 0 < k < L the cycle with the fast
    diagonalization equals the one with the dense coarse solve; whole solves
    meet the tolerance against the dense full solve."""
    m = omesh.Mesh.box((3, 2, 3), 8, 1.0, 1.2)          # levels 2, 4, 8
    cs = CondensedSystem(m)
    r = synth.random_grid(m.shape, 5) * m.free_skeleton_mask()
    top = solver.Hierarchy(m, coarse="fd", coarse_level=2)
    assert top.L == 0
    ref = cs.to_grid(np.linalg.solve(cs.Hhat, cs.to_vec(r)))
    assert np.linalg.norm(top.vcycle(None, r) - ref) <= 1e-12 * np.linalg.norm(ref)
    a = solver.Hierarchy(m, coarse="fd", coarse_level=1).vcycle(None, r)
    b = solver.Hierarchy(m, exact_coarse=True, coarse_level=1).vcycle(None, r)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(a - ref) > 1e-6 * np.linalg.norm(ref)    # one smoothed level left
    f = synth.random_grid(m.shape, 6)
    res = solver.solve(m, f, rtol=1e-11, coarse="fd", coarse_level=1)
    full = cs.full_solve(m.assembled_mass() * f)
    assert np.linalg.norm(res.u - full) <= 1e-9 * np.linalg.norm(full)
    with pytest.raises(ValueError):
        solver.Hierarchy(m, coarse_level=1)                   # coarse CG: level 0 only
    with pytest.raises(ValueError):
        solver.Hierarchy(m, coarse="fd", coarse_level=3)
