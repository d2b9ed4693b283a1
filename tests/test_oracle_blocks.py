"""Pins of the oracle's element-centred block smoother (Sec. 3.4) against
plain definitions: the dense block operator R_e Hhat R_e^T solved by LU,
the full-block fast diagonalization, the exact condensed solve when one
block covers the whole mesh, the 1D eigen identities with identity padding,
and the partition of unity of the block weights."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import blocks, sem1d
from oracle import mesh as omesh
from oracle.dense import CondensedSystem, block_nodes, block_smoother_matrix

MESHES = [
    # (n, p, lambda, alpha): interior and boundary blocks, one element in a
    # direction, stretched widths, lambda = 0
    ((3, 3, 3), 2, 1.0, 1.3),
    ((4, 3, 2), 3, 0.0, 1.0),
    ((2, 2, 2), 4, 1.0, 1.2),
    ((1, 2, 3), 3, 2.0, 1.0),
]


@pytest.fixture(scope="module")
def systems():
    return {c: CondensedSystem(omesh.Mesh.box(c[0], c[1], c[2], c[3])) for c in MESHES}


@pytest.mark.parametrize("case", MESHES)
@pytest.mark.parametrize("weights", ["smooth", "mult"])
def test_block_smoother_equals_dense_definition(systems, case, weights):
    """sum_e W_e R_e^T (R_e Hhat R_e^T)^-1 R_e r with dense LU per block,
    against the six-face algorithm and against the full-block fast
    diagonalization."""
    cs = systems[case]
    m = cs.mesh
    r = synth.random_grid(m.shape, 1) * m.free_skeleton_mask()
    S = block_smoother_matrix(cs, 0.7, weights)
    ref = cs.to_grid(S @ cs.to_vec(r))
    for route in ("tpc", "tpf"):
        got = blocks.block_smoother(m, r, 0.7, route, weights)
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref), (route, weights)


@pytest.mark.parametrize("case", MESHES)
def test_block_weights_partition_of_unity(systems, case):
    cs = systems[case]
    m = cs.mesh
    tot = np.zeros(int(np.prod(m.shape)))
    for e3 in range(m.n[2]):
        for e2 in range(m.n[1]):
            for e1 in range(m.n[0]):
                e = (e1, e2, e3)
                g, offs = block_nodes(cs, e)
                w = [blocks.block_weights_1d(m.n[d], m.p, e[d]) for d in range(3)]
                np.add.at(tot, g, w[0][offs[:, 0]] * w[1][offs[:, 1]] * w[2][offs[:, 2]])
    assert np.max(np.abs(tot[cs.B] - 1.0)) <= 1e-14


def test_block_weights_interior_values():
    """Away from the boundary the 1D weight is q(t)/2, 1/2, q(1-t)/2 on the
    block's left, centre and right element (q(t) = 35t^4 - 84t^5 + 70t^6 -
    20t^7): at the block's two face positions 1/2, at the centre element's
    nodes 1/2, at the left element's first interior node q(t_1)/2."""
    p, n = 5, 7
    x, _ = sem1d.gll(p)
    w = blocks.block_weights_1d(n, p, 3)
    assert abs(w[p - 1] - 0.5) < 1e-15 and abs(w[2 * p - 1] - 0.5) < 1e-15
    assert np.allclose(w[p:2 * p - 1], 0.5, atol=1e-15)
    t = (x[1] + 1.0) / 2.0
    q = 35 * t ** 4 - 84 * t ** 5 + 70 * t ** 6 - 20 * t ** 7
    assert abs(w[0] - q / 2.0) < 1e-15
    assert abs(w[3 * p - 2] - q / 2.0) < 1e-15       # mirror image at the right end


@pytest.mark.parametrize("p", [2, 4, 7])
def test_single_element_block_is_the_exact_solve(p):
    """On one element the block of that element is the whole mesh (its
    neighbours are ghosts): the smoother is the exact condensed solve
    Hhat^-1 r with weight one."""
    m = omesh.Mesh.box((1, 1, 1), p, 1.5, 1.0, lengths=(1.0, 2.0, 0.7))
    cs = CondensedSystem(m)
    r = synth.random_grid(m.shape, 3) * m.free_skeleton_mask()
    ref = cs.to_grid(np.linalg.solve(cs.Hhat, cs.to_vec(r)))
    got = blocks.block_smoother(m, r, 1.0)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("e", [0, 2, 4])
def test_block_tables_1d_eigen_identities(e):
    """S^T M S = I and S^T L S = diag(lam) on the coupled positions of the
    assembled 3-element block, identity padding (eigenvalue 1) on ghost and
    Dirichlet positions."""
    p = 4
    hs = synth.stretched_widths(5, 1.3)
    S, lam, coupled = blocks.block_tables_1d(hs, p, e)
    nS = 3 * p - 1
    M = np.zeros(3 * p + 1)
    L = np.zeros((3 * p + 1, 3 * p + 1))
    for j, el in enumerate((e - 1, e, e + 1)):
        if 0 <= el < len(hs):
            me, Le = sem1d.element_matrices(p, hs[el])
            M[j * p:(j + 1) * p + 1] += me
            L[j * p:(j + 1) * p + 1, j * p:(j + 1) * p + 1] += Le
    M, L = M[1:3 * p], L[1:3 * p, 1:3 * p]
    c = np.flatnonzero(coupled)
    Sc = S[np.ix_(c, c)]
    assert np.allclose(Sc.T @ np.diag(M[c]) @ Sc, np.eye(len(c)), atol=1e-12)
    assert np.allclose(Sc.T @ L[np.ix_(c, c)] @ Sc, np.diag(lam[c]), atol=1e-10 * lam.max())
    d = np.flatnonzero(~coupled)
    assert np.array_equal(S[np.ix_(d, d)], np.eye(len(d))) and np.all(lam[d] == 1.0)
    assert not S[np.ix_(c, d)].any() and not S[np.ix_(d, c)].any()
    if e == 0:      # ghost left element (positions 0..p-2) and the Dirichlet vertex p-1
        assert not coupled[:p].any() and coupled[p:].all()
    assert len(coupled) == nS
