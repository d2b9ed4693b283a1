"""Pins of the oracle's 1D building blocks against textbook facts.

GLL nodes/weights for small p in closed form, quadrature exactness,
stiffness energy identities, generalized eigenpairs, interpolation and the
degree-7 weight polynomial of Sec. 3.2.
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


def _blocks_1d(p):
    """The 1D problems whose eigenpairs the method uses at degree p: the
    element interior (p - 1 nodes) and a star's two-element block with the
    two outer ends removed (2p - 1 nodes), here with unequal widths."""
    m, L = sem1d.element_matrices(p, 0.37)
    yield "interior", L[1:p, 1:p], m[1:p]
    M = np.zeros(2 * p + 1)
    LL = np.zeros((2 * p + 1, 2 * p + 1))
    for k, h in enumerate((0.37, 0.37 * 1.35)):
        mk, Lk = sem1d.element_matrices(p, h)
        M[k * p:k * p + p + 1] += mk
        LL[k * p:k * p + p + 1, k * p:k * p + p + 1] += Lk
    yield "star", LL[1:2 * p, 1:2 * p], M[1:2 * p]


def _sturm_counts(L, m, shifts, dps=30):
    """Number of eigenvalues of the pencil (L, diag m) below each shift,
    exactly up to 30-digit rounding: Householder reduction of
    m^-1/2 L m^-1/2 to tridiagonal form in mpmath, then Sylvester's law of
    inertia through the Sturm sequence of the tridiagonal matrix."""
    import mpmath
    mp = mpmath.mp
    old = mp.dps
    mp.dps = dps
    try:
        n = len(m)
        sq = [mpmath.sqrt(mpmath.mpf(float(x))) for x in m]
        A = [[mpmath.mpf(float(L[i, j])) / (sq[i] * sq[j]) for j in range(n)] for i in range(n)]
        for k in range(n - 2):                       # Householder: zero A[k+2:, k]
            alpha = mpmath.sqrt(mpmath.fsum(A[i][k] ** 2 for i in range(k + 1, n)))
            if alpha == 0:
                continue
            if A[k + 1][k] > 0:
                alpha = -alpha
            v = [mpmath.mpf(0)] * n
            for i in range(k + 1, n):
                v[i] = A[i][k]
            v[k + 1] -= alpha
            beta = 2 / mpmath.fsum(t * t for t in v)
            # A <- (I - beta v v^T) A (I - beta v v^T) = A - v q^T - q v^T
            pv = [beta * mpmath.fsum(A[i][j] * v[j] for j in range(k + 1, n)) for i in range(n)]
            K = beta * mpmath.fsum(v[i] * pv[i] for i in range(k + 1, n)) / 2
            q = [pv[i] - K * v[i] for i in range(n)]
            for i in range(n):
                for j in range(n):
                    if v[i] != 0 or v[j] != 0:
                        A[i][j] -= v[i] * q[j] + q[i] * v[j]
        a = [A[i][i] for i in range(n)]
        b2 = [A[i + 1][i] * A[i][i + 1] for i in range(n - 1)]
        out = []
        for s in shifts:
            s = mpmath.mpf(s)
            cnt, q = 0, a[0] - s
            cnt += q < 0
            for i in range(1, n):
                q = a[i] - s - b2[i - 1] / q
                cnt += q < 0
            out.append(cnt)
        return out
    finally:
        mp.dps = old


@pytest.mark.parametrize("p", [16, 32, 48])
def test_generalized_eigenvalues_exact_to_1e14(p):
    """Every eigenvalue of gen_eig at large p lies within a relative 1e-14 of
    the true eigenvalue of the same index: Sturm counts (30 digits) just
    below and just above each one differ by exactly one and equal its
    index.  An FP64 eigensolver misses this bound at p = 32 and 48 (its
    smallest star eigenvalues are off by up to ~4e-12 relative)."""
    delta = 1e-14
    for name, L, m in _blocks_1d(p):
        S, lam = sem1d.gen_eig(L, np.diag(m))
        shifts = [x for l in lam for x in (l * (1 - delta), l * (1 + delta))]
        cnt = _sturm_counts(L, m, shifts)
        assert cnt == [i + k for i in range(len(lam)) for k in (0, 1)], name


@pytest.mark.parametrize("p", [16, 48])
def test_generalized_eigenvectors_high_precision(p):
    """S^T M S = I and S^T L S = diag(lam) evaluated at 30 digits (so that
    the check is not itself limited by FP64 sums): the eigenvectors are the
    M-orthonormal eigenvectors of the pencil to FP64 rounding of S."""
    import mpmath
    mpmath.mp.dps = 30
    for name, L, m in _blocks_1d(p):
        S, lam = sem1d.gen_eig(L, np.diag(m))
        n = len(m)
        Sm = mpmath.matrix(S.tolist())
        Lm = mpmath.matrix(L.tolist())
        Mm = mpmath.diag([mpmath.mpf(float(x)) for x in m])
        G = Sm.T * Mm * Sm
        K = Sm.T * Lm * Sm
        lmax = float(lam.max())
        for i in range(n):
            for j in range(n):
                gij = float(G[i, j]) - (1.0 if i == j else 0.0)
                kij = float(K[i, j]) - (float(lam[i]) if i == j else 0.0)
                assert abs(gij) <= 1e-14, (name, i, j, gij)
                assert abs(kij) <= 1e-14 * lmax, (name, i, j, kij)
