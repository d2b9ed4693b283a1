"""Pins of the oracle's inhomogeneous-Dirichlet route (lifting).

The lifted solve must reproduce, at every node and to rounding, any
polynomial solution the discrete space holds exactly: GLL quadrature with
p + 1 points integrates degree 2p - 1 exactly, so for u linear (p >= 1), u a
harmonic quadratic (p >= 2) or u cubic with its Laplacian in f (p >= 3) the
Galerkin equations hold for the nodal interpolant of u itself (the lumped
mass enters both sides the same way).  A wrong sign, index or scale in the
lift breaks these by O(1).  The lift is also checked against the dense
partition H_fD g_D and against its homogeneous special case, and the full
solve against spectral convergence on a trigonometric solution.
"""
import numpy as np
import pytest

from oracle import dense, dirichlet, mesh as M


def _mesh(n, p, lam, alpha):
    return M.Mesh.box(n, p, lam, alpha=alpha, lengths=(1.0, 1.3, 0.8))


def _fields(mesh, kind, lam):
    """(u, f) with f = lam u - Laplacian(u) on the node grid."""
    X3, X2, X1 = mesh.coords()
    one = np.ones(mesh.shape)
    if kind == "linear":
        u = (0.3 + 1.1 * X1 - 0.7 * X2 + 0.4 * X3) * one
        lap = 0.0 * one
    elif kind == "harmonic2":
        u = (X1 ** 2 - X2 ** 2 + X1 * X3 - 0.5 * X2) * one
        lap = 0.0 * one
    else:  # cubic
        u = (X1 ** 3 + X2 * X3 ** 2 - 0.5 * X3 + 2.0) * one
        lap = (6.0 * X1 + 2.0 * X2) * one
    return u, lam * u - lap


EXACT = [("linear", 1), ("linear", 2), ("harmonic2", 2), ("harmonic2", 3), ("cubic", 3), ("cubic", 4)]


@pytest.mark.parametrize("lam", [0.0, 2.5])
@pytest.mark.parametrize("kind,p", EXACT)
def test_polynomial_solutions_reproduced(kind, p, lam):
    mesh = _mesh((2, 3, 2), p, lam, 1.4)
    u, f = _fields(mesh, kind, lam)
    ue = dirichlet.exact_solve(mesh, f, u)
    assert np.max(np.abs(ue - u)) < 1e-11 * max(1.0, np.max(np.abs(u)))
    res = dirichlet.solve(mesh, f, u, rtol=1e-13, coarse_rtol=1e-14)
    assert np.max(np.abs(res.u - u)) < 1e-10 * max(1.0, np.max(np.abs(u)))


def test_lift_matches_dense_partition():
    mesh = _mesh((2, 3, 2), 3, 0.7, 1.3)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(mesh.shape)
    g = rng.standard_normal(mesh.shape)
    H = dense.assemble_H(mesh)
    D = mesh.dirichlet_mask().ravel()
    fr = ~D
    Mf = mesh.assembled_mass().ravel()
    want = f.ravel().copy()
    want[fr] -= (H[np.ix_(fr, D)] @ g.ravel()[D]) / Mf[fr]
    want[D] = 0.0
    got = dirichlet.lift_rhs(mesh, f, g).ravel()
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_lift_ignores_interior_data_and_reduces_to_homogeneous():
    mesh = _mesh((3, 2, 2), 2, 1.0, 1.0)
    rng = np.random.default_rng(6)
    f = rng.standard_normal(mesh.shape)
    D = mesh.dirichlet_mask()
    g = np.where(D, 0.0, rng.standard_normal(mesh.shape))   # interior entries only
    np.testing.assert_array_equal(dirichlet.lift_rhs(mesh, f, g), np.where(D, 0.0, f))


def test_lift_touches_only_nodes_next_to_the_boundary():
    mesh = _mesh((4, 4, 4), 2, 1.0, 1.0)
    rng = np.random.default_rng(7)
    g = rng.standard_normal(mesh.shape)
    d = dirichlet.lift_rhs(mesh, np.zeros(mesh.shape), g)
    p = mesh.p
    inner = d[p + 1:-p - 1, p + 1:-p - 1, p + 1:-p - 1]   # nodes outside the boundary elements
    assert np.all(inner == 0.0)
    assert np.count_nonzero(d) > 0


def test_spectral_convergence_trig_solution():
    errs = []
    for p in (2, 4, 6):
        mesh = M.Mesh.box((2, 2, 2), p, 0.0, lengths=(2 * np.pi, 2 * np.pi, 2 * np.pi))
        X3, X2, X1 = mesh.coords()
        a = (0.6, 0.5, 0.4)
        u = np.sin(a[0] * X1 + 0.3) * np.sin(a[1] * X2 + 0.7) * np.sin(a[2] * X3 + 1.1)
        f = (a[0] ** 2 + a[1] ** 2 + a[2] ** 2) * u
        res = dirichlet.solve(mesh, f, u, rtol=1e-12)
        errs.append(np.max(np.abs(res.u - u)))
    assert errs[0] > 20 * errs[1] > 400 * errs[2]
    assert errs[2] < 1e-5


def test_paper_test_solution_generator():
    """The manufactured solution of Sec. 5.2: the plane-wave sum equals the
    product of the five factors, and its Laplacian matches a fourth-order
    finite-difference Laplacian at random points."""
    import synth
    rng = np.random.default_rng(8)
    x = rng.uniform(0.0, 2 * np.pi, size=(3, 50))
    for k in (1.0, 5.0):
        u, f = synth.paper_test_solution(k, 0.0, x[0], x[1], x[2])
        prod = (np.cos(k * (x[0] - 3 * x[1] + 2 * x[2])) * np.sin(k * (1 + x[0]))
                * np.sin(k * (1 - x[1])) * np.sin(k * (2 * x[0] + x[1]))
                * np.sin(k * (3 * x[0] - 2 * x[1] + 2 * x[2])))
        assert np.max(np.abs(u - prod)) < 1e-13
        h = 1e-3 / k
        lap = 0.0
        for d in range(3):
            def at(s):
                y = x.copy()
                y[d] += s * h
                return synth.paper_test_solution(k, 0.0, y[0], y[1], y[2])[0]
            lap = lap + (-at(2) + 16 * at(1) - 30 * u + 16 * at(-1) - at(-2)) / (12 * h * h)
        assert np.max(np.abs(-lap - f)) < 1e-6 * np.max(np.abs(f))
        _, f2 = synth.paper_test_solution(k, 3.0, x[0], x[1], x[2])
        assert np.allclose(f2, 3.0 * u + f, rtol=0, atol=1e-12 * np.max(np.abs(f)))
