"""Matrix-free operators of the condensed system (oracle, FP64 by default).

Condensed vectors are stored as full node grids (N3, N2, N1) whose entries
at element-interior and Dirichlet nodes are zero; plain sums over the grid
are therefore sums over the unique condensed unknowns.

Passages followed:
* condensed operator Hhat_e u_B = H_BB u_B - H_BI H_II^-1 H_IB u_B
  (Sec. 2.2), with H_II^-1 applied by fast diagonalization of the element
  interior (Sec. 3.2, eq. fast_diagonalization); written out as the
  definition, O(p^4) per element, not the paper's cited O(p^3) form;
* star inverse, Alg. 1 (Sec. 3.2) -- the tensor-product inverse in the
  condensed system (TPC) -- together with the full-star fast
  diagonalization (TPF, eq. fast_diagonalization) as a second route;
* Schwarz smoother, Alg. 2 with the weight functions of Sec. 3.2 and the
  boundary treatment by identity padding of Sec. 3.3;
* grid transfers: embedded tensor-product interpolation restricted to the
  condensed system, restriction = transpose (Sec. 4.1);
* static condensation of the right-hand side and interior recovery
  (Alg. 4, first and last steps).
"""
from __future__ import annotations

import numpy as np

from . import sem1d
from .mesh import Mesh


# --------------------------------------------------------------------------
# batched tensor helpers; element arrays are (E, n3, n2, n1)
# --------------------------------------------------------------------------
def _ax1(A, u):
    """Apply batched matrices A (E, out, in) along the last (x1) axis."""
    return np.matmul(u, np.swapaxes(A, 1, 2)[:, None])


def _ax2(A, u):
    return np.matmul(A[:, None], u)


def _ax3(A, u):
    E, n3, n2, n1 = u.shape
    return np.matmul(A, u.reshape(E, n3, n2 * n1)).reshape(E, A.shape[1], n2, n1)


def _apply_He(u, m1, m2, m3, L1, L2, L3, lam):
    """Element operator eq. (helmholtzop) on a batch of element arrays."""
    M3 = m3[:, :, None, None]
    M2 = m2[:, None, :, None]
    M1 = m1[:, None, None, :]
    y = lam * M3 * M2 * M1 * u
    y = y + M3 * M2 * _ax1(L1, u)
    y = y + M3 * M1 * _ax2(L2, u)
    y = y + M2 * M1 * _ax3(L3, u)
    return y


class ElementTables:
    """Per direction and element index: 1D mass, stiffness, interior eigenpairs."""

    def __init__(self, mesh: Mesh):
        p = mesh.p
        self.p = p
        self.m, self.L, self.S, self.lam = [], [], [], []
        for d in range(3):
            ms, Ls, Ss, ls = [], [], [], []
            for h in mesh.h[d]:
                m, L = sem1d.element_matrices(p, h)
                ms.append(m)
                Ls.append(L)
                if p >= 2:
                    S, lam = sem1d.gen_eig(L[1:p, 1:p], np.diag(m[1:p]))
                else:
                    S, lam = np.zeros((0, 0)), np.zeros(0)
                Ss.append(S)
                ls.append(lam)
            self.m.append(np.array(ms))
            self.L.append(np.array(Ls))
            self.S.append(np.array(Ss))
            self.lam.append(np.array(ls))


class _Elements:
    """Gathered per-element tables for a mesh (cached on the mesh object)."""

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        t = ElementTables(mesh)
        idx, e1, e2, e3 = mesh.element_index_arrays()
        self.idx = idx
        self.m = [t.m[0][e1], t.m[1][e2], t.m[2][e3]]
        self.L = [t.L[0][e1], t.L[1][e2], t.L[2][e3]]
        self.S = [t.S[0][e1], t.S[1][e2], t.S[2][e3]]
        self.l = [t.lam[0][e1], t.lam[1][e2], t.lam[2][e3]]
        p = mesh.p
        inner = np.zeros((p + 1,) * 3, dtype=bool)
        if p >= 2:
            inner[1:p, 1:p, 1:p] = True
        self.inner = inner
        self.free = mesh.free_skeleton_mask()

    def He(self, u):
        return _apply_He(u, *self.m, *self.L, self.mesh.lam)

    def HII_inv(self, w):
        """H_II^-1 w by fast diagonalization of the element interior."""
        S1, S2, S3 = self.S
        l1, l2, l3 = self.l
        t = _ax1(np.swapaxes(S1, 1, 2), w)
        t = _ax2(np.swapaxes(S2, 1, 2), t)
        t = _ax3(np.swapaxes(S3, 1, 2), t)
        D = (self.mesh.lam + l3[:, :, None, None] + l2[:, None, :, None]
             + l1[:, None, None, :])
        t = t / D
        t = _ax1(S1, t)
        t = _ax2(S2, t)
        return _ax3(S3, t)

    def gather(self, grid):
        return np.asarray(grid).ravel()[self.idx]

    def scatter(self, ye):
        N = int(np.prod(self.mesh.shape))
        return np.bincount(self.idx.ravel(), weights=ye.ravel(),
                           minlength=N).reshape(self.mesh.shape)


def _elements(mesh: Mesh) -> _Elements:
    cache = getattr(mesh, "_oracle_elements", None)
    if cache is None:
        cache = _Elements(mesh)
        mesh._oracle_elements = cache
    return cache


def condensed_op(mesh: Mesh, u_grid):
    """y = Hhat u on the condensed unknowns (Sec. 2.2), assembled."""
    el = _elements(mesh)
    p = mesh.p
    u = el.gather(u_grid)
    u = np.where(el.inner[None], 0.0, u)
    y1 = el.He(u)
    if p >= 2:
        w = y1[:, 1:p, 1:p, 1:p]
        v = np.zeros_like(u)
        v[:, 1:p, 1:p, 1:p] = el.HII_inv(w)
        y2 = el.He(v)
        ye = y1 - y2
    else:
        ye = y1
    ye = np.where(el.inner[None], 0.0, ye)
    y = el.scatter(ye)
    return np.where(el.free, y, 0.0)


def condense_rhs(mesh: Mesh, f_grid):
    """Fhat = F_B - H_BI H_II^-1 F_I with F = M f (GLL-lumped mass)."""
    el = _elements(mesh)
    p = mesh.p
    F = mesh.assembled_mass() * np.asarray(f_grid)
    Fhat = np.where(el.free, F, 0.0)
    if p >= 2:
        Fe = el.gather(F)
        v = np.zeros_like(Fe)
        v[:, 1:p, 1:p, 1:p] = el.HII_inv(Fe[:, 1:p, 1:p, 1:p])
        corr = el.He(v)
        corr = np.where(el.inner[None], 0.0, corr)
        Fhat = Fhat - np.where(el.free, el.scatter(corr), 0.0)
    return Fhat


def recover_interior(mesh: Mesh, f_grid, uhat_grid):
    """u = (uhat, H_II^-1 (F_I - H_IB uhat)) on the full node grid (Alg. 4)."""
    el = _elements(mesh)
    p = mesh.p
    u = np.where(el.free, np.asarray(uhat_grid), 0.0)
    if p < 2:
        return mesh.expand_periodic(u)
    F = mesh.assembled_mass() * np.asarray(f_grid)
    ue = el.gather(u)
    ue = np.where(el.inner[None], 0.0, ue)
    w = el.gather(F)[:, 1:p, 1:p, 1:p] - el.He(ue)[:, 1:p, 1:p, 1:p]
    uI = el.HII_inv(w)
    out = u.ravel().copy()
    out[el.idx[:, 1:p, 1:p, 1:p].ravel()] = uI.ravel()
    return mesh.expand_periodic(out.reshape(mesh.shape))


# --------------------------------------------------------------------------
# stars (Sec. 3)
# --------------------------------------------------------------------------
def star_tables_1d(hs, p, v, bc=("D", "D")):
    """1D star matrices for vertex index v on the element widths ``hs``.

    The 2-element block around the vertex is assembled on positions -p..p,
    the outer ends +-p are dropped (homogeneous local problem), leaving
    n_S = 2p-1 positions.  Sec. 3.3: positions outside the domain (ghost
    element beyond a Dirichlet or Neumann side) are decoupled, and so is a
    Dirichlet vertex: S = identity and eigenvalue 1 there, the eigenpairs of
    the remaining block fill the rest.  A Neumann vertex stays coupled; in a
    periodic direction the ghost element is element n-1 (v = 0) and nothing
    is decoupled.  Returns (S, lam, coupled mask) with S^T M S = I,
    S^T L S = diag(lam) on the coupled block.
    """
    n = len(hs)
    nS = 2 * p - 1
    per = bc[0] == "P"
    M = np.zeros(2 * p + 1)
    L = np.zeros((2 * p + 1, 2 * p + 1))
    coupled = np.zeros(2 * p + 1, dtype=bool)
    if v >= 1 or per:
        m, Le = sem1d.element_matrices(p, hs[(v - 1) % n])
        M[0:p + 1] += m
        L[0:p + 1, 0:p + 1] += Le
        coupled[0:p + 1] = True
    if v <= n - 1:
        m, Le = sem1d.element_matrices(p, hs[v])
        M[p:2 * p + 1] += m
        L[p:2 * p + 1, p:2 * p + 1] += Le
        coupled[p:2 * p + 1] = True
    if (v == 0 and bc[0] == "D") or (v == n and bc[1] == "D"):
        coupled[p] = False          # Dirichlet vertex
    M, L, coupled = M[1:2 * p], L[1:2 * p, 1:2 * p], coupled[1:2 * p]
    S = np.eye(nS)
    lam = np.ones(nS)
    c = np.flatnonzero(coupled)
    if len(c):
        Sc, lc = sem1d.gen_eig(L[np.ix_(c, c)], np.diag(M[c]))
        S[np.ix_(c, c)] = Sc
        lam[c] = lc
    return S, lam, coupled


def star_inverse_tpc(F1, F2, F3, S1, S2, S3, l1, l2, l3, lam):
    """Alg. 1: solution on the three star faces from the face residuals.

    Batched over stars (leading axis).  F1[i3, i2] lies on the face normal
    to x1, F2[i3, i1] normal to x2, F3[i2, i1] normal to x3; index p-1 is
    the star vertex.  The faces carry duplicated copies of the three axis
    lines and the vertex; step 1 divides them by their multiplicity.
    """
    nS = F1.shape[-1]
    c = (nS - 1) // 2
    mult = np.ones((nS, nS))
    mult[c, :] += 1.0
    mult[:, c] += 1.0
    mult[c, c] = 3.0
    F1, F2, F3 = F1 / mult, F2 / mult, F3 / mult
    T = np.swapaxes
    # 2D transforms into the eigenspace of each face
    G1 = T(S3, 1, 2) @ F1 @ S2          # (k3, k2)
    G2 = T(S3, 1, 2) @ F2 @ S1          # (k3, k1)
    G3 = T(S2, 1, 2) @ F3 @ S1          # (k2, k1)
    a1, a2, a3 = S1[:, c, :], S2[:, c, :], S3[:, c, :]
    # expansion into the 3D star eigenspace and the inverse eigenvalues
    E = (a1[:, None, None, :] * G1[:, :, :, None]
         + a2[:, None, :, None] * G2[:, :, None, :]
         + a3[:, :, None, None] * G3[:, None, :, :])
    D = (lam + l1[:, None, None, :] + l2[:, None, :, None]
         + l3[:, :, None, None])
    V = E / D
    # contraction back onto each face and the 2D back transforms
    H1 = np.einsum("sabk,sk->sab", V, a1)
    H2 = np.einsum("sakb,sk->sab", V, a2)
    H3 = np.einsum("skab,sk->sab", V, a3)
    U1 = S3 @ H1 @ T(S2, 1, 2)
    U2 = S3 @ H2 @ T(S1, 1, 2)
    U3 = S2 @ H3 @ T(S1, 1, 2)
    return U1, U2, U3


def star_inverse_tpf(F1, F2, F3, S1, S2, S3, l1, l2, l3, lam):
    """Full-star fast diagonalization (TPF) restricted to the faces.

    The face residual (each node once) is placed in the full n_S^3 block,
    mapped by (S^T x S^T x S^T), scaled by D^-1 and mapped back by
    (S x S x S) (eq. fast_diagonalization); the faces are then read off.
    """
    nS = F1.shape[-1]
    c = (nS - 1) // 2
    ns = F1.shape[0]
    R = np.zeros((ns, nS, nS, nS))          # [i3, i2, i1]
    R[:, :, :, c] = F1
    m2 = np.ones((nS, nS), dtype=bool)
    m2[:, c] = False
    R[:, :, c, :] = np.where(m2, F2, R[:, :, c, :])
    m3 = np.ones((nS, nS), dtype=bool)
    m3[c, :] = False
    m3[:, c] = False
    R[:, c, :, :] = np.where(m3, F3, R[:, c, :, :])
    T = np.swapaxes
    t = _ax1(T(S1, 1, 2), R)
    t = _ax2(T(S2, 1, 2), t)
    t = _ax3(T(S3, 1, 2), t)
    D = (lam + l1[:, None, None, :] + l2[:, None, :, None]
         + l3[:, :, None, None])
    t = t / D
    t = _ax1(S1, t)
    t = _ax2(S2, t)
    u = _ax3(S3, t)
    return u[:, :, :, c], u[:, :, c, :], u[:, c, :, :]


class _Stars:
    """Star index maps and gathered 1D star tables for a mesh."""

    def __init__(self, mesh: Mesh, pw: int = 7):
        self.mesh = mesh
        p = mesh.p
        nS = 2 * p - 1
        n1, n2, n3 = mesh.n
        N1, N2, N3 = mesh.N
        # one star per vertex; in a periodic direction vertex n_d is vertex 0
        nv = [mesh.n[d] + (0 if mesh.periodic[d] else 1) for d in range(3)]
        tabs = []
        for d in range(3):
            Ss, ls = [], []
            for v in range(nv[d]):
                S, lam, _ = star_tables_1d(mesh.h[d], p, v, mesh.bc[d])
                Ss.append(S)
                ls.append(lam)
            tabs.append((np.array(Ss), np.array(ls)))
        v3, v2, v1 = np.meshgrid(np.arange(nv[2]), np.arange(nv[1]),
                                 np.arange(nv[0]), indexing="ij")
        v1, v2, v3 = v1.ravel(), v2.ravel(), v3.ravel()
        self.v = (v1, v2, v3)
        self.S = [tabs[0][0][v1], tabs[1][0][v2], tabs[2][0][v3]]
        self.l = [tabs[0][1][v1], tabs[1][1][v2], tabs[2][1][v3]]
        off = np.arange(nS) - (p - 1)
        sentinel = N1 * N2 * N3
        self.sentinel = sentinel

        def flat(i1, i2, i3):
            i1, i2, i3 = mesh.wrap(0, i1), mesh.wrap(1, i2), mesh.wrap(2, i3)
            ok = ((i1 >= 0) & (i1 < N1) & (i2 >= 0) & (i2 < N2)
                  & (i3 >= 0) & (i3 < N3))
            return np.where(ok, (i3 * N2 + i2) * N1 + i1, sentinel)

        c1, c2, c3 = v1 * p, v2 * p, v3 * p
        A = off[None, :, None]
        B = off[None, None, :]
        # F1[i3, i2] at x1 = c1, F2[i3, i1] at x2 = c2, F3[i2, i1] at x3 = c3
        self.idx1 = flat(c1[:, None, None], c2[:, None, None] + B,
                         c3[:, None, None] + A)
        self.idx2 = flat(c1[:, None, None] + B, c2[:, None, None],
                         c3[:, None, None] + A)
        self.idx3 = flat(c1[:, None, None] + B, c2[:, None, None] + A,
                         c3[:, None, None])
        w1 = sem1d.star_weights_1d(p, pw)
        self.W1 = np.broadcast_to(w1[:, None] * w1[None, :], (nS, nS))
        c = p - 1
        keep2 = np.ones((nS, nS), dtype=bool)
        keep2[:, c] = False
        keep3 = np.ones((nS, nS), dtype=bool)
        keep3[c, :] = False
        keep3[:, c] = False
        self.keep = (np.ones((nS, nS), dtype=bool), keep2, keep3)
        self.free = mesh.free_skeleton_mask().ravel()


def _stars(mesh: Mesh) -> _Stars:
    cache = getattr(mesh, "_oracle_stars", None)
    if cache is None:
        cache = _Stars(mesh)
        mesh._oracle_stars = cache
    return cache


def smoother(mesh: Mesh, r_grid, omega: float = 1.0, route: str = "tpc",
             chunk: int = 4096):
    """Alg. 2: du = omega sum_i W_i R_i^T Hhat_i^-1 Mhat_i^-1 R_i r.

    ``route`` selects the star inverse: "tpc" (Alg. 1) or "tpf".  Stars are
    processed in chunks to bound memory.
    """
    st = _stars(mesh)
    p = mesh.p
    if p < 1:
        raise ValueError
    r = np.append(np.asarray(r_grid, dtype=np.float64).ravel(), 0.0)
    r = np.where(np.append(st.free, False), r, 0.0)
    nstars = st.idx1.shape[0]
    N = st.sentinel
    du = np.zeros(N + 1)
    inv = star_inverse_tpc if route == "tpc" else star_inverse_tpf
    for s0 in range(0, nstars, chunk):
        sl = slice(s0, min(nstars, s0 + chunk))
        F = [r[st.idx1[sl]], r[st.idx2[sl]], r[st.idx3[sl]]]
        U = inv(F[0], F[1], F[2], st.S[0][sl], st.S[1][sl], st.S[2][sl],
                st.l[0][sl], st.l[1][sl], st.l[2][sl], mesh.lam)
        for Uf, idx, keep in zip(U, (st.idx1, st.idx2, st.idx3), st.keep):
            ii = idx[sl]
            vals = np.where(keep[None], Uf * st.W1[None], 0.0)
            du += np.bincount(ii.ravel(), weights=vals.ravel(), minlength=N + 1)
    du = du[:N]
    du = np.where(st.free, du, 0.0)
    return omega * du.reshape(mesh.shape)


# --------------------------------------------------------------------------
# grid transfers (Sec. 4.1)
# --------------------------------------------------------------------------
def _interp_1d(hs, pc, pf, periodic=False):
    """Element-wise Lagrange interpolation from degree pc to pf along one
    direction (rows fine nodes, columns coarse nodes).  Periodic: the last
    coarse node is the first one, so its column is added to the first, and
    the last fine node (a mirror) gets no row."""
    n = len(hs)
    xc, _ = sem1d.gll(pc)
    xf, _ = sem1d.gll(pf)
    J = sem1d.lagrange_matrix(xc, xf)
    P = np.zeros((n * pf + 1, n * pc + 1))
    for e in range(n):
        P[e * pf: e * pf + pf + 1, e * pc: e * pc + pc + 1] = J
    if periodic:
        P[:, 0] += P[:, -1]
        P[:, -1] = 0.0
        P[-1, :] = 0.0
    return P


def prolong(mesh_c: Mesh, mesh_f: Mesh, uc_grid):
    """Fine condensed values = 3D tensor interpolation of the coarse ones."""
    P = [_interp_1d(mesh_c.h[d], mesh_c.p, mesh_f.p, mesh_c.periodic[d]) for d in range(3)]
    u = np.where(mesh_c.free_skeleton_mask(), np.asarray(uc_grid), 0.0)
    u = np.einsum("ia,cba->cbi", P[0], u, optimize=True)
    u = np.einsum("ib,cba->cia", P[1], u, optimize=True)
    u = np.einsum("ic,cba->iba", P[2], u, optimize=True)
    return np.where(mesh_f.free_skeleton_mask(), u, 0.0)


def restrict(mesh_f: Mesh, mesh_c: Mesh, rf_grid):
    """Exact transpose of ``prolong`` on the condensed unknowns."""
    P = [_interp_1d(mesh_c.h[d], mesh_c.p, mesh_f.p, mesh_c.periodic[d]) for d in range(3)]
    r = np.where(mesh_f.free_skeleton_mask(), np.asarray(rf_grid), 0.0)
    r = np.einsum("ia,cbi->cba", P[0], r, optimize=True)
    r = np.einsum("ib,cia->cba", P[1], r, optimize=True)
    r = np.einsum("ic,iba->cba", P[2], r, optimize=True)
    return np.where(mesh_c.free_skeleton_mask(), r, 0.0)


# --------------------------------------------------------------------------
# h-transfers between degree-1 meshes (coarse-grid multigrid below p_0)
# --------------------------------------------------------------------------
def merged_widths(hs):
    """Element widths of the mesh with pairs of neighbouring elements merged."""
    hs = np.asarray(hs, dtype=np.float64)
    if len(hs) % 2:
        raise ValueError("even element count required")
    return hs[0::2] + hs[1::2]


def _h_interp_1d(hf):
    """Linear interpolation from the vertices of the merged mesh to the
    vertices of the mesh with widths ``hf`` (rows fine, columns coarse)."""
    nf = len(hf)
    P = np.zeros((nf + 1, nf // 2 + 1))
    for i in range(nf + 1):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            t = hf[i - 1] / (hf[i - 1] + hf[i])
            P[i, (i - 1) // 2] = 1.0 - t
            P[i, (i + 1) // 2] = t
    return P


def h_prolong(mesh_c: Mesh, mesh_f: Mesh, uc_grid):
    """Trilinear interpolation of degree-1 nodal values from the merged mesh
    (homogeneous Dirichlet boundaries only)."""
    assert mesh_c.p == 1 and mesh_f.p == 1
    if not (mesh_c.all_dirichlet() and mesh_f.all_dirichlet()):
        raise NotImplementedError("degree-1 h-levels: Dirichlet boundaries only")
    P = [_h_interp_1d(mesh_f.h[d]) for d in range(3)]
    u = np.where(mesh_c.free_skeleton_mask(), np.asarray(uc_grid), 0.0)
    u = np.einsum("ia,cba->cbi", P[0], u, optimize=True)
    u = np.einsum("ib,cba->cia", P[1], u, optimize=True)
    u = np.einsum("ic,cba->iba", P[2], u, optimize=True)
    return np.where(mesh_f.free_skeleton_mask(), u, 0.0)


def h_restrict(mesh_f: Mesh, mesh_c: Mesh, rf_grid):
    """Exact transpose of ``h_prolong``."""
    if not (mesh_c.all_dirichlet() and mesh_f.all_dirichlet()):
        raise NotImplementedError("degree-1 h-levels: Dirichlet boundaries only")
    P = [_h_interp_1d(mesh_f.h[d]) for d in range(3)]
    r = np.where(mesh_f.free_skeleton_mask(), np.asarray(rf_grid), 0.0)
    r = np.einsum("ia,cbi->cba", P[0], r, optimize=True)
    r = np.einsum("ib,cia->cba", P[1], r, optimize=True)
    r = np.einsum("ic,iba->cba", P[2], r, optimize=True)
    return np.where(mesh_c.free_skeleton_mask(), r, 0.0)


# --------------------------------------------------------------------------
# diagonal of the condensed operator (coarse-grid Jacobi preconditioner)
# --------------------------------------------------------------------------
def condensed_diagonal(mesh: Mesh):
    """diag(Hhat) assembled from element-wise probing with unit vectors."""
    el = _elements(mesh)
    p = mesh.p
    shell = np.argwhere(~el.inner)
    E = el.idx.shape[0]
    diag_e = np.zeros((E, p + 1, p + 1, p + 1))
    for (a, b, c) in shell:
        u = np.zeros((E, p + 1, p + 1, p + 1))
        u[:, a, b, c] = 1.0
        y1 = el.He(u)
        if p >= 2:
            v = np.zeros_like(u)
            v[:, 1:p, 1:p, 1:p] = el.HII_inv(y1[:, 1:p, 1:p, 1:p])
            y = y1 - el.He(v)
        else:
            y = y1
        diag_e[:, a, b, c] = y[:, a, b, c]
    d = el.scatter(diag_e)
    return np.where(el.free, d, 1.0)
