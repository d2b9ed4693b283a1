"""Pins of the oracle's 1D building blocks against textbook facts.

GLL nodes/weights for small p in closed form, quadrature exactness,
stiffness energy identities, generalized eigenpairs, interpolation and the
degree-7 weight polynomial of Sec. 3.3.
"""
import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from oracle import sem1d


def test_gll_closed_forms():
    x, w = sem1d.gll(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = sem1d.gll(3)
    assert np.allclose(x, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w = sem1d.gll(4)
    assert np.allclose(x, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 13, 16, 32, 48])
def test_gll_quadrature_exactness(p):
    x, w = sem1d.gll(p)
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.all(np.diff(x) > 0)
    for k in range(2 * p):                       # exact up to degree 2p-1
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13
    if 2 <= p <= 8:                              # not exact at degree 2p
        assert abs(np.dot(w, x ** (2 * p)) - 2 / (2 * p + 1)) > 1e-6


@pytest.mark.parametrize("p", [2, 4, 7, 12])
def test_stiffness_energy_and_derivative(p):
    x, w = sem1d.gll(p)
    D = sem1d.diff_matrix(x)
    w_, L = sem1d.standard_matrices(p)
    rng = np.random.default_rng(p)
    assert np.max(np.abs(L @ np.ones(p + 1))) < 1e-12 * p * p
    assert np.max(np.abs(L - L.T)) < 1e-12 * p * p
    for _ in range(3):
        c = rng.standard_normal(p + 1)           # polynomial of degree p
        u = P.polyval(x, c)
        du = P.polyder(c)
        assert np.allclose(D @ u, P.polyval(x, du), atol=1e-10 * p * p)
        energy = P.polyint(P.polymul(du, du))
        exact = P.polyval(1.0, energy) - P.polyval(-1.0, energy)
        assert abs(u @ L @ u - exact) < 1e-10 * max(1.0, abs(exact))


def test_element_scaling():
    m, L = sem1d.element_matrices(4, 0.25)
    w, Ls = sem1d.standard_matrices(4)
    assert np.allclose(m, 0.125 * w) and np.allclose(L, 8.0 * Ls)


@pytest.mark.parametrize("p", [3, 8])
def test_generalized_eigenpairs(p):
    m, L = sem1d.element_matrices(p, 0.7)
    Li, Mi = L[1:p, 1:p], np.diag(m[1:p])
    S, lam = sem1d.gen_eig(Li, Mi)
    assert np.allclose(S.T @ Mi @ S, np.eye(p - 1), atol=1e-12)
    assert np.allclose(S.T @ Li @ S, np.diag(lam), atol=1e-10 * lam.max())


def test_low_eigenvalues_approach_dirichlet_laplacian():
    # 1D Dirichlet problem on [0, 1] with 6 elements of degree 8: the lowest
    # generalized eigenvalues approximate (k pi)^2 spectrally
    n, p = 6, 8
    N = n * p + 1
    M = np.zeros(N)
    L = np.zeros((N, N))
    for e in range(n):
        m, Le = sem1d.element_matrices(p, 1.0 / n)
        M[e * p:e * p + p + 1] += m
        L[e * p:e * p + p + 1, e * p:e * p + p + 1] += Le
    S, lam = sem1d.gen_eig(L[1:-1, 1:-1], np.diag(M[1:-1]))
    k = np.arange(1, 6)
    assert np.allclose(lam[:5], (k * np.pi) ** 2, rtol=1e-9)


@pytest.mark.parametrize("pc,pf", [(2, 4), (4, 8), (3, 12)])
def test_interpolation_reproduces_polynomials(pc, pf):
    xc, _ = sem1d.gll(pc)
    xf, _ = sem1d.gll(pf)
    J = sem1d.lagrange_matrix(xc, xf)
    c = np.random.default_rng(0).standard_normal(pc + 1)
    assert np.allclose(J @ P.polyval(xc, c), P.polyval(xf, c), atol=1e-13)
    assert np.allclose(J.sum(axis=1), 1.0, atol=1e-14)


def test_weight_polynomial():
    c = sem1d.weight_poly_coeffs(7)
    assert np.array_equal(c, [0, 0, 0, 0, 35, -84, 70, -20])
    t = np.linspace(0, 1, 101)
    q = sem1d.weight_poly(t)
    assert np.allclose(q + sem1d.weight_poly(1 - t), 1.0, atol=1e-14)   # partition of unity
    for der in (1, 2, 3):
        dc = P.polyder(c, der)
        assert abs(P.polyval(0.0, dc)) < 1e-12 and abs(P.polyval(1.0, dc)) < 1e-12
    assert sem1d.weight_poly(1.0) == 1.0 and sem1d.weight_poly(0.0) == 0.0
    w = sem1d.star_weights_1d(5)
    assert w[4] == 1.0 and np.allclose(w, w[::-1]) and np.all(np.diff(w[:5]) > 0)
