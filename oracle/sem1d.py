"""One-dimensional spectral-element building blocks (oracle, FP64).

Paper passages followed:
* Sec. 2.1, eq. (helmholtzop) and the d_e coefficients: GLL mass matrix M
  (diagonal, GLL quadrature) and stiffness matrix L of the standard element;
  on an element of width h the physical matrices are (h/2) M and (2/h) L.
* Sec. 3.2 (fast diagonalization): generalized eigenpairs S^T L S = Lambda,
  S^T M S = I.
* Sec. 3.2 (weight functions): polynomials of degree p_W that are one at the
  star vertex, zero at the other vertex and have vanishing higher
  derivatives there (p_W = 7 in the paper).
* Sec. 4.1: interpolation between polynomial degrees for the p-multigrid.

All routines are written from the textbook definitions (Lagrange
polynomials, Gauss-Lobatto quadrature); they are deliberately unoptimised.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def legendre(p: int, x):
    """P_p(x) and P_{p-1}(x) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if p == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, p + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p1, p0


def gll(p: int):
    """Gauss-Lobatto-Legendre nodes and weights on [-1, 1], p >= 1.

    Nodes are -1, 1 and the roots of P_p'.  Interior roots are found by
    Newton's method on P_p' using the Legendre differential equation
    (1-x^2) P'' = 2x P' - p(p+1) P, started from Chebyshev-Lobatto points.
    Weights: w_i = 2 / (p (p+1) P_p(x_i)^2).
    """
    if p < 1:
        raise ValueError("p >= 1 required")
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    inner = x[1:-1].copy()
    for _ in range(100):
        P, Pm1 = legendre(p, inner)
        dP = p * (Pm1 - inner * P) / (1.0 - inner ** 2)
        d2P = (2.0 * inner * dP - p * (p + 1) * P) / (1.0 - inner ** 2)
        step = dP / d2P
        inner -= step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    x[1:-1] = inner
    x[0], x[-1] = -1.0, 1.0
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P ** 2)
    return x, w


def lagrange_matrix(xfrom, xto):
    """J[i, j] = l_j(xto[i]) for the Lagrange basis on the nodes ``xfrom``."""
    xfrom = np.asarray(xfrom, dtype=np.float64)
    xto = np.asarray(xto, dtype=np.float64)
    n = len(xfrom)
    J = np.ones((len(xto), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                J[:, j] *= (xto - xfrom[m]) / (xfrom[j] - xfrom[m])
    return J


def diff_matrix(x):
    """D[i, j] = l_j'(x_i) from the barycentric form of the Lagrange basis."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    lam = np.array([1.0 / np.prod([x[j] - x[m] for m in range(n) if m != j])
                    for j in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def standard_matrices(p: int):
    """Standard-element GLL mass (diagonal, returned as vector) and stiffness.

    M_S = diag(w);  L_S[i, j] = sum_q w_q l_i'(x_q) l_j'(x_q) = (D^T M_S D).
    GLL quadrature with p+1 points is exact to degree 2p-1, so L_S is exact.
    """
    x, w = gll(p)
    D = diff_matrix(x)
    L = D.T @ np.diag(w) @ D
    # L is symmetric by definition; the FP64 product is so only to ~1e-14,
    # and eigen solvers read one triangle of it
    return w, 0.5 * (L + L.T)


def element_matrices(p: int, h: float):
    """Physical 1D mass (vector) and stiffness on an element of width h."""
    w, L = standard_matrices(p)
    return 0.5 * h * w, (2.0 / h) * L


def _two_sum(a, b):
    """s + e = a + b exactly (Knuth's TwoSum)."""
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _two_prod(a, b):
    """x + e = a b exactly (Dekker's TwoProduct, 64-bit significand)."""
    f = np.longdouble(4294967297.0)          # 2^32 + 1 splits a longdouble
    x = a * b
    c = f * a
    ah = c - (c - a)
    al = a - ah
    c = f * b
    bh = c - (c - b)
    bl = b - bh
    return x, al * bl - (((x - ah * bh) - al * bh) - ah * bl)


def _matmul2(A, B):
    """A @ B with every entry summed as if in twice the working precision
    (compensated dot product, Dot2 of Ogita, Rump & Oishi 2005)."""
    S = np.zeros((A.shape[0], B.shape[1]), dtype=A.dtype)
    C = np.zeros_like(S)
    for k in range(A.shape[1]):
        p, pe = _two_prod(A[:, k, None], B[None, k, :])
        S, se = _two_sum(S, p)
        C = C + (pe + se)
    return S + C


def gen_eig(L, M):
    """S, lam with S^T L S = diag(lam), S^T M S = I (M diagonal, positive).

    The pairs are those of the symmetric A = M^-1/2 L M^-1/2 (S = M^-1/2 Q).
    Route: a LAPACK eigendecomposition of A in FP64, then iterative
    refinement of the whole decomposition by the method of Ogita & Aishima
    (2018) in extended precision (numpy longdouble).  One step maps an
    approximate eigenvector matrix X to X (I + E), where, with R = I - X^T X
    and T = X^T A X, the eigenvalue estimates are t_ii / (1 - r_ii) and E
    has diagonal r_ii / 2 and off-diagonal (t_ij + lam_j r_ij) /
    (lam_j - lam_i); the error contracts quadratically.  Pairs whose
    estimates lie within delta = 2 (||T - diag(lam)|| + ||A|| ||R||) of each
    other are treated as one cluster, E_ij = r_ij / 2 (the same paper's rule
    for multiple eigenvalues: periodic 1D problems have double ones), which
    only re-orthonormalises the basis of the cluster.  The last step and
    the final Rayleigh quotients form R and T with compensated products, so
    that the small eigenvalues (~p^-4 of the largest at large p) come out
    with relative, not only absolute, accuracy; an FP64 solver alone leaves
    them with relative errors up to ~1e-11.
    """
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    m = np.diag(M)
    if not np.array_equal(M, np.diag(m)):
        raise ValueError("gen_eig expects a diagonal M")
    n = L.shape[0]
    X = np.longdouble
    ms = np.sqrt(m.astype(X))
    A = L.astype(X) / (ms[:, None] * ms[None, :])
    _, Q0 = scipy.linalg.eigh(A.astype(np.float64))
    Q = Q0.astype(X)
    eye = np.eye(n, dtype=X)
    for step in range(3):
        mm = _matmul2 if step == 2 else np.matmul
        R = eye - mm(Q.T, Q)
        T = mm(Q.T, mm(A, Q))
        lam = np.diag(T) / (1 - np.diag(R))
        gap = lam[None, :] - lam[:, None]            # lam_j - lam_i
        np.fill_diagonal(gap, 1)
        delta = 2 * (np.linalg.norm((T - np.diag(lam)).astype(np.float64), 2)
                     + np.linalg.norm(A.astype(np.float64), 2) * np.linalg.norm(R.astype(np.float64), 2))
        near = np.abs(gap) <= delta
        E = np.where(near, R / 2, (T + lam[None, :] * R) / np.where(near, 1, gap))
        np.fill_diagonal(E, np.diag(R) / 2)
        Q = Q + Q @ E
    AQ = _matmul2(A, Q)
    lam = np.array([_matmul2(Q[:, i:i + 1].T, AQ[:, i:i + 1])[0, 0]
                    / _matmul2(Q[:, i:i + 1].T, Q[:, i:i + 1])[0, 0] for i in range(n)])
    order = np.argsort(lam)
    S = Q[:, order] / ms[:, None]
    return S.astype(np.float64), lam[order].astype(np.float64)


def weight_poly_coeffs(pw: int = 7):
    """Monomial coefficients c[k] of q(t) = sum c_k t^k, degree pw (odd).

    q(1) = 1 (star vertex), q(0) = 0 (the other vertex) and the first
    (pw-1)/2 derivatives vanish at both ends.  The (pw+1) x (pw+1) system of
    these conditions is solved exactly in rational arithmetic.
    """
    from fractions import Fraction
    from math import factorial
    if pw < 1 or pw % 2 == 0:
        raise ValueError("odd p_W required")
    nd = (pw - 1) // 2
    rows = []
    for t0, val in ((0, 0), (1, 1)):
        for der in range(nd + 1):
            row = [Fraction(0)] * (pw + 1)
            for k in range(der, pw + 1):
                row[k] = Fraction(factorial(k), factorial(k - der)) * \
                    Fraction(t0) ** (k - der)
            rows.append(row + [Fraction(val if der == 0 else 0)])
    n = pw + 1
    for col in range(n):                       # Gauss-Jordan, exact
        piv = next(r for r in range(col, n) if rows[r][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        pv = rows[col][col]
        rows[col] = [x / pv for x in rows[col]]
        for r in range(n):
            if r != col and rows[r][col] != 0:
                f = rows[r][col]
                rows[r] = [a - f * b for a, b in zip(rows[r], rows[col])]
    return np.array([float(rows[k][n]) for k in range(n)])


def weight_poly(t, pw: int = 7):
    c = weight_poly_coeffs(pw)
    t = np.asarray(t, dtype=np.float64)
    return sum(ck * t ** k for k, ck in enumerate(c))


def star_weights_1d(p: int, pw: int = 7):
    """1D star weights at offsets -(p-1)..(p-1) from the star vertex.

    A node at offset j lies at reference coordinate xi_{|j|} of the element
    on that side; its distance parameter towards the vertex is
    t = (1 - xi_{|j|}) / 2, which is 1 at the vertex and 0 at the far vertex.
    """
    x, _ = gll(p)
    off = np.arange(-(p - 1), p)
    return weight_poly((1.0 - x[np.abs(off)]) / 2.0, pw)
