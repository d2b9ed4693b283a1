"""Pins of the oracle's Neumann and periodic boundaries (Sec. 3.3).

The boundary kinds enter the oracle in four places: the node masks, the
element-to-node map (wrapping in a periodic direction), the 1D star and
fast-diagonalization tables (ghost elements decoupled, a Neumann vertex kept
coupled) and the transfers (the mirror column folded).  Each is pinned
against something that does not share its construction:

* counts of unknowns in closed form;
* constants in the kernel of the assembled operator at lambda = 0 (a wrong
  wrap or a missing element leaves a row sum nonzero);
* the matrix-free routes against dense plain definitions on tiny meshes
  (Schur complement, inverted principal submatrices for the stars, the 3D
  interpolation matrix with the mirror columns folded node by node);
* manufactured solutions that satisfy the boundary conditions exactly, whose
  discrete solutions converge spectrally in p;
* translation invariance of the periodic problem on a uniform mesh.
"""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import coarse_fd, dense, matfree, solver
from oracle import mesh as M

# (n, p, lambda, alpha, bc)
TINY = [
    ((3, 2, 2), 3, 1.0, 1.0, ("P", "N", "D")),
    ((2, 3, 2), 2, 0.5, 1.3, (("N", "D"), "P", ("D", "N"))),
    ((3, 3, 2), 3, 1.0, 1.0, ("P", "P", "N")),
    ((2, 2, 2), 4, 2.0, 1.2, ("N", "N", "N")),
    ((3, 2, 3), 1, 1.0, 1.0, ("P", ("D", "N"), "P")),
    ((2, 2, 3), 3, 0.0, 1.4, (("D", "N"), "N", "P")),
]


def _ids(c):
    bc = "".join(b if isinstance(b, str) else "".join(b) for b in c[4])
    return f"n{''.join(map(str, c[0]))}-p{c[1]}-{bc}"


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def systems():
    cache = {}

    def get(case):
        if case not in cache:
            n, p, lam, a, bc = case
            m = M.Mesh.box(n, p, lam, a, bc=bc)
            cache[case] = (m, dense.CondensedSystem(m))
        return cache[case]
    return get


def test_parse_and_reject():
    assert M.parse_bc("DNPPDD") == (("D", "N"), ("P", "P"), ("D", "D"))
    assert M.parse_bc(None) == (("D", "D"),) * 3
    with pytest.raises(ValueError):
        M.parse_bc((("P", "D"), "D", "D"))
    with pytest.raises(ValueError):
        M.Mesh.box((3, 3, 3), 2, 0.0, bc=("N", "P", "N"))      # singular
    with pytest.raises(ValueError):
        M.Mesh.box((2, 3, 3), 2, 1.0, bc=("P", "D", "D"))      # periodic, 2 elements


@pytest.mark.parametrize("case", TINY, ids=_ids)
def test_unknown_counts(case):
    """Per direction the unknown node indices are N_d minus one per
    Dirichlet side, minus the mirror layer if periodic; the condensed system
    has all of them except the n_e (p-1)^3 element interiors."""
    n, p, lam, a, bc = case
    m = M.Mesh.box(n, p, lam, a, bc=bc)
    u = []
    for d in range(3):
        lo, hi = m.bc[d]
        u.append(m.N[d] - (lo == "D") - (hi == "D") - (lo == "P"))
    assert int(m.free_mask().sum()) == u[0] * u[1] * u[2]
    assert int(m.free_skeleton_mask().sum()) == u[0] * u[1] * u[2] - m.n_elements() * (p - 1) ** 3


@pytest.mark.parametrize("bc", [("P", "P", "P"), ("N", "N", "N"), ("P", "N", "P")])
def test_constants_in_the_kernel(bc):
    """lambda = 0 without a Dirichlet side: H 1 = 0 on the unknowns, and
    the condensed operator annihilates the constant skeleton vector."""
    m = M.Mesh.box((3, 3, 3), 3, 1.0, 1.25, bc=bc)
    m0 = M.Mesh(m.h[0], m.h[1], m.h[2], m.p, 1.0, bc)
    m0.lam = 0.0                      # bypass the singularity check on purpose
    H = dense.assemble_H(m0)
    free = m0.free_mask().ravel()
    one = free.astype(float)
    assert np.max(np.abs((H @ one)[free])) < 1e-11 * np.abs(H).max()
    y = matfree.condensed_op(m0, m0.free_skeleton_mask().astype(float))
    assert np.max(np.abs(y)) < 1e-11 * np.abs(H).max()


@pytest.mark.parametrize("case", TINY, ids=_ids)
def test_condensed_operator_matches_dense(systems, case):
    m, cs = systems(case)
    for seed in (1, 2):
        u = synth.random_grid(m.shape, seed) * m.free_skeleton_mask()
        ref = cs.to_grid(cs.Hhat @ cs.to_vec(u))
        assert rel(matfree.condensed_op(m, u), ref) < 1e-12


@pytest.mark.parametrize("case", TINY, ids=_ids)
def test_condensation_and_recovery_match_dense(systems, case):
    m, cs = systems(case)
    f = m.expand_periodic(synth.random_grid(m.shape, 3))
    F = m.assembled_mass() * f
    Fh = matfree.condense_rhs(m, f)
    assert rel(cs.to_vec(Fh), cs.condense_rhs(F)) < 1e-12
    uhat = np.linalg.solve(cs.Hhat, cs.to_vec(Fh))
    u = matfree.recover_interior(m, f, cs.to_grid(uhat))
    full = cs.full_solve(F)
    assert rel(u, full) < 1e-11
    # mirror entries repeat the first layer
    assert np.array_equal(u, m.expand_periodic(u))


@pytest.mark.parametrize("case", TINY, ids=_ids)
@pytest.mark.parametrize("route", ["tpc", "tpf"])
def test_star_smoother_matches_dense(systems, case, route):
    """Alg. 2 with identity-padded boundary stars (Sec. 3.3) equals the sum
    of weighted inverses of the principal submatrices of Hhat on the star
    nodes (eq. smoother_definition)."""
    m, cs = systems(case)
    S = cs.smoother_matrix(omega=0.7)
    r = synth.random_grid(m.shape, 5) * m.free_skeleton_mask()
    ref = cs.to_grid(S @ cs.to_vec(r))
    assert rel(matfree.smoother(m, r, omega=0.7, route=route), ref) < 1e-11


@pytest.mark.parametrize("case", TINY, ids=_ids)
def test_star_weights_partition_of_unity(systems, case):
    """The unit-weight-free check: with every star inverse replaced by the
    identity the weights sum to 1 at every unknown."""
    m, cs = systems(case)
    w1 = __import__("oracle.sem1d", fromlist=["x"]).star_weights_1d(m.p)
    tot = np.zeros(len(cs.B))
    for v in cs.vertices():
        g, offs = cs.star_nodes(v)
        k = np.array([cs.pos[x] for x in g], dtype=np.int64)
        if len(k):
            tot[k] += (w1[offs[:, 0] + m.p - 1] * w1[offs[:, 1] + m.p - 1]
                       * w1[offs[:, 2] + m.p - 1])
    assert np.allclose(tot, 1.0, atol=1e-13)


@pytest.mark.parametrize("case", [c for c in TINY if c[1] >= 2], ids=_ids)
def test_transfers_match_dense(case):
    n, p, lam, a, bc = case
    mf = M.Mesh.box(n, 2 * p, lam, a, bc=bc)
    mc = mf.with_degree(p)
    P = dense.prolongation_matrix(mc, mf)
    cf = dense.CondensedSystem(mf)
    cc = dense.CondensedSystem(mc)
    uc = synth.random_grid(mc.shape, 6) * mc.free_skeleton_mask()
    assert rel(cf.to_vec(matfree.prolong(mc, mf, uc)), P @ cc.to_vec(uc)) < 1e-13
    rf = synth.random_grid(mf.shape, 7) * mf.free_skeleton_mask()
    assert rel(cc.to_vec(matfree.restrict(mf, mc, rf)), P.T @ cf.to_vec(rf)) < 1e-13


def test_prolongation_reproduces_periodic_interpolant():
    """Coarse nodal values of a smooth periodic function: the prolonged
    values at the fine skeleton nodes equal the element-wise degree-pc
    interpolant evaluated there (computed here directly per element)."""
    mc = M.Mesh.box((3, 3, 3), 3, 1.0, 1.0, lengths=(2 * np.pi, 1.0, 1.0), bc=("P", "N", "N"))
    mf = mc.with_degree(6)
    X3, X2, X1 = mc.coords()
    uc = np.sin(X1) * np.cos(np.pi * X2) * (1 + X3) + 0 * X3
    uc = uc * mc.free_skeleton_mask()
    uf = matfree.prolong(mc, mf, uc)
    # direct: separable interpolation per element along each direction
    from oracle import sem1d
    xc, _ = sem1d.gll(3)
    xf, _ = sem1d.gll(6)
    J = sem1d.lagrange_matrix(xc, xf)
    Uc = np.sin(X1) * np.cos(np.pi * X2) * (1 + X3) + 0 * X3
    ref = np.zeros(mf.shape)
    for e3 in range(3):
        for e2 in range(3):
            for e1 in range(3):
                blk = Uc[e3 * 3:e3 * 3 + 4, e2 * 3:e2 * 3 + 4, e1 * 3:e1 * 3 + 4]
                blk = np.einsum("ia,cba->cbi", J, blk)
                blk = np.einsum("ib,cba->cia", J, blk)
                blk = np.einsum("ic,cba->iba", J, blk)
                ref[e3 * 6:e3 * 6 + 7, e2 * 6:e2 * 6 + 7, e1 * 6:e1 * 6 + 7] = blk
    mask = mf.free_skeleton_mask()
    assert np.max(np.abs(np.where(mask, uf - ref, 0.0))) < 1e-13


@pytest.mark.parametrize("case", TINY, ids=_ids)
def test_fd_solves_match_dense(systems, case):
    m, cs = systems(case)
    F = synth.random_grid(m.shape, 8) * m.free_skeleton_mask()
    ref = cs.to_grid(np.linalg.solve(cs.Hhat, cs.to_vec(F)))
    assert rel(coarse_fd.fd_condensed_solve(m, F), ref) < 1e-12
    Ff = synth.random_grid(m.shape, 9) * m.free_mask()
    assert rel(coarse_fd.fd_solve_full(m, Ff), cs.full_solve(Ff)) < 1e-12


def _manufactured(bc_kind):
    """Exact solutions on (0, 2 pi) x (0, 1) x (0, 1) meeting the boundary
    kinds: sin(x1 + 0.3) is 2 pi periodic, cos(pi x) has zero slope at both
    ends, sin(pi x / 2) vanishes at 0 with zero slope at 1, cos(pi x / 2)
    has zero slope at 0 and vanishes at 1, sin(pi x) vanishes at both."""
    f1 = {"P": (lambda x: np.sin(x + 0.3), 1.0)}
    f = {("N", "N"): (lambda x: np.cos(np.pi * x), np.pi ** 2),
         ("D", "N"): (lambda x: np.sin(np.pi * x / 2), np.pi ** 2 / 4),
         ("N", "D"): (lambda x: np.cos(np.pi * x / 2), np.pi ** 2 / 4),
         ("D", "D"): (lambda x: np.sin(np.pi * x), np.pi ** 2)}
    return f1["P"], f[bc_kind[0]], f[bc_kind[1]]


@pytest.mark.parametrize("kinds", [(("N", "N"), ("D", "N")), (("N", "D"), ("N", "N")),
                                   (("D", "D"), ("N", "D"))])
def test_manufactured_solution_converges_spectrally(kinds):
    (g1, k1), (g2, k2), (g3, k3) = _manufactured(kinds)
    lam = 1.0
    errs = []
    for p in (4, 8):
        m = M.Mesh.box((3, 2, 2), p, lam, 1.0, lengths=(2 * np.pi, 1.0, 1.0),
                       bc=("P", kinds[0], kinds[1]))
        X3, X2, X1 = m.coords()
        u = g1(X1) * g2(X2) * g3(X3)
        f = (k1 + k2 + k3 + lam) * u
        res = solver.solve(m, f, method="kMG", rtol=1e-12, coarse="fd")
        assert res.iters <= 12
        errs.append(np.max(np.abs(res.u - u)))
    assert errs[1] < 2e-6 and errs[1] < 1e-2 * errs[0], errs


def test_periodic_translation_invariance():
    """Uniform periodic mesh: shifting the data by one element along the
    periodic direction shifts the discrete solution by the same amount."""
    m = M.Mesh.box((4, 3, 3), 4, 1.0, 1.0, bc=("P", "N", ("D", "N")))
    p = m.p
    f = m.expand_periodic(synth.random_grid(m.shape, 10))
    fs = np.roll(f[:, :, :-1], p, axis=2)
    fs = m.expand_periodic(np.concatenate([fs, fs[:, :, :1]], axis=2))
    a = solver.solve(m, f, rtol=1e-13, coarse="fd").u
    b = solver.solve(m, fs, rtol=1e-13, coarse="fd").u
    a_s = np.roll(a[:, :, :-1], p, axis=2)
    assert rel(b[:, :, :-1], a_s) < 1e-10


@pytest.mark.parametrize("case", [c for c in TINY if c[1] >= 2], ids=_ids)
def test_vcycle_fd_equals_dense_coarse(case):
    n, p, lam, a, bc = case
    m = M.Mesh.box(n, 2 * p, lam, a, bc=bc)
    r = synth.random_grid(m.shape, 11) * m.free_skeleton_mask()
    x = solver.Hierarchy(m, coarse="fd").vcycle(None, r)
    y = solver.Hierarchy(m, exact_coarse=True).vcycle(None, r)
    assert rel(x, y) < 1e-11


def test_unsupported_combinations_raise():
    m = M.Mesh.box((4, 4, 4), 4, 1.0, bc=("P", "N", "D"))
    with pytest.raises(NotImplementedError):
        solver.Hierarchy(m, hmg_levels=1)


@pytest.mark.parametrize("case", [c for c in TINY if c[1] >= 2], ids=_ids)
@pytest.mark.parametrize("route", ["tpc", "tpf"])
def test_block_smoother_matches_dense(systems, case, route):
    """The element-centred blocks of Sec. 3.4 with the boundary treatment of
    Sec. 3.3 (ghost elements and Dirichlet vertices identity-padded, a
    periodic block continuing across the seam) equal the weighted inverses
    of the principal submatrices of Hhat on the block nodes."""
    from oracle import blocks
    m, cs = systems(case)
    S = dense.block_smoother_matrix(cs, omega=0.9)
    r = synth.random_grid(m.shape, 13) * m.free_skeleton_mask()
    ref = cs.to_grid(S @ cs.to_vec(r))
    assert rel(blocks.block_smoother(m, r, omega=0.9, route=route), ref) < 1e-11


@pytest.mark.parametrize("case", [c for c in TINY if c[1] >= 2], ids=_ids)
def test_block_weights_partition_of_unity(systems, case):
    m, cs = systems(case)
    from oracle.blocks import block_weights_1d
    tot = np.zeros(len(cs.B))
    for e3 in range(m.n[2]):
        for e2 in range(m.n[1]):
            for e1 in range(m.n[0]):
                g, offs = dense.block_nodes(cs, (e1, e2, e3))
                k = np.array([cs.pos[x] for x in g], dtype=np.int64)
                w = [block_weights_1d(m.n[d], m.p, (e1, e2, e3)[d], periodic=m.periodic[d]) for d in range(3)]
                tot[k] += w[0][offs[:, 0]] * w[1][offs[:, 1]] * w[2][offs[:, 2]]
    assert np.allclose(tot, 1.0, atol=1e-13)


def test_block_smoother_solve_with_seams():
    """ipCG with the element-centred smoother on a mesh with every kind of
    side reaches the manufactured solution's discrete solution."""
    m = M.Mesh.box((3, 3, 3), 6, 1.0, 1.2, bc=("P", ("N", "D"), "N"))
    f = synth.random_grid(m.shape, 14)
    a = solver.solve(m, f, rtol=1e-11, coarse="fd", smoother="element")
    b = solver.solve(m, f, rtol=1e-11, coarse="fd")
    assert rel(a.u, b.u) < 1e-9
    assert a.iters <= b.iters
