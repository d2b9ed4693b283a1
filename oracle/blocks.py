"""Element-centred block smoother (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU baseline use this package; the product path never does.

Passages followed (Sec. 3.4, "Extension to element-centered block
smoothers"): the subdomain of element e is the block of 3 x 3 x 3 elements
centred on it (full overlap of one element in every direction).  In the
residual form the block's outer boundary is homogeneous, leaving
n_S = 3p - 1 positions per direction; after static condensation the block
keeps the six faces of its centre element, each extended over the block
(an n_S x n_S window of the element-boundary plane).  The block operator
keeps the tensor-product form of eq. helmholtzop with the 1D matrices
restricted to the block, so the block inverse is the star algorithm of
Alg. 1 with six faces instead of three: 2D transforms of every face into the
1D eigenbases, expansion into the 3D eigenspace with the rows of the
eigenvector matrices at the two face positions of each direction, the
inverse eigenvalue sums, contraction back onto the six faces and the 2D back
transforms (73 n_S^3 operations).  The boundary treatment is that of
Sec. 3.3: ghost elements and Dirichlet vertices are decoupled by identity
padding of the 1D eigenvector matrices (eigenvalue 1) and a zero right-hand
side there.  The corrections are combined as in eq. smoother_definition.

Readings (the paper is silent on them):
* weights: the paper names inverse multiplicity weighting as one that needs
  no relaxation and distance-based weights as better; here the 1D block
  weight is the distance-based one built from the degree-7 weight polynomial
  q of the star smoother: q(t)/2 on the left element, 1/2 on the centre
  element, q(1-t)/2 on the right element (t the element reference
  coordinate in [0, 1]), which sums to one over the three blocks covering a
  point; near the domain boundary, where a covering block is missing, the
  present blocks' weights are divided by their sum.  ``weights="mult"``
  gives the inverse multiplicity instead.  The 3D weight is the product of
  the 1D ones (the blocks covering a node are the product of the 1D sets);
* every element of the mesh centres one block (blocks of boundary elements
  reach into ghost elements, which are decoupled).
"""
from __future__ import annotations

import numpy as np

from . import sem1d
from .mesh import Mesh


def block_tables_1d(hs, p, e, bc=("D", "D")):
    """1D matrices of the block of element e on the element widths ``hs``.

    Elements e-1, e, e+1 are assembled on positions 0..3p and the outer ends
    0 and 3p are dropped, leaving n_S = 3p - 1 positions.  Positions inside a
    ghost element and Dirichlet boundary vertices are decoupled: S =
    identity and eigenvalue 1 there; the eigenpairs of the coupled block
    fill the rest (Sec. 3.3: a Neumann vertex stays coupled; in a periodic
    direction the neighbours of the end elements wrap round and nothing is
    decoupled).  Returns (S, lam, coupled) with S^T M S = I and
    S^T L S = diag(lam) on the coupled positions.
    """
    n = len(hs)
    nS = 3 * p - 1
    per = bc[0] == "P"
    M = np.zeros(3 * p + 1)
    L = np.zeros((3 * p + 1, 3 * p + 1))
    coupled = np.zeros(3 * p + 1, dtype=bool)
    for j, el in enumerate((e - 1, e, e + 1)):
        if per:
            el %= n
        if 0 <= el <= n - 1:
            m, Le = sem1d.element_matrices(p, hs[el])
            sl = slice(j * p, (j + 1) * p + 1)
            M[sl] += m
            L[sl, sl] += Le
            coupled[sl] = True
    if e == 0 and bc[0] == "D":
        coupled[p] = False          # the domain boundary x = 0 (Dirichlet)
    if e == n - 1 and bc[1] == "D":
        coupled[2 * p] = False      # the domain boundary x = end (Dirichlet)
    M, L, coupled = M[1:3 * p], L[1:3 * p, 1:3 * p], coupled[1:3 * p]
    S = np.eye(nS)
    lam = np.ones(nS)
    c = np.flatnonzero(coupled)
    if len(c):
        Sc, lc = sem1d.gen_eig(L[np.ix_(c, c)], np.diag(M[c]))
        S[np.ix_(c, c)] = Sc
        lam[c] = lc
    return S, lam, coupled


def _phi(n, p, x_ref, eb, g, pw, periodic=False):
    """Unnormalised distance weight of the block of element eb at global
    position g (valid only where the block covers g)."""
    m, j = divmod(g, p)                     # g lies in element m at local node j
    if m >= n:                              # the last grid point: t = 1 of element n-1
        m, j = n - 1, p
    t = (x_ref[j] + 1.0) / 2.0
    rel = (m - eb) % n if periodic else m - eb
    if rel == 0:
        return 0.5
    if rel == -1 or (periodic and rel == n - 1):   # the block's left element
        return 0.5 * float(sem1d.weight_poly(t, pw))
    if rel == 1:                            # the block's right element
        return 0.5 * float(sem1d.weight_poly(1.0 - t, pw))
    return 0.0


def block_weights_1d(n, p, e, weights="smooth", pw=7, periodic=False):
    """1D weights of the block of element e at its n_S positions (global
    node index g = (e-1) p + 1 + o for position o, modulo n p in a periodic
    direction), on n elements.

    Summed over all blocks of the mesh that cover a node they give one.
    """
    nS = 3 * p - 1
    x_ref, _ = sem1d.gll(p)
    w = np.zeros(nS)
    for o in range(nS):
        g = (e - 1) * p + 1 + o
        if periodic:
            g %= n * p
            cover = [b for b in range(n) if 0 < (g - (b - 1) * p) % (n * p) < 3 * p]
        else:
            if g < 0 or g > n * p:
                continue
            cover = [b for b in range(n) if (b - 1) * p < g < (b + 2) * p]
        if e not in cover:
            continue
        if weights == "mult":
            w[o] = 1.0 / len(cover)
        else:
            # at an element boundary the node is t = 1 of the left element
            # and t = 0 of the right one; the weight functions are continuous
            tot = sum(_phi(n, p, x_ref, b, g, pw, periodic) for b in cover)
            w[o] = _phi(n, p, x_ref, e, g, pw, periodic) / tot
    return w


def face_multiplicity(nS, cs):
    """Copies of each face node among the six gathered faces: 1, plus one for
    each in-plane coordinate that lies on a face position of its direction."""
    on = np.zeros(nS, dtype=bool)
    on[list(cs)] = True
    return 1.0 + on[:, None].astype(float) + on[None, :].astype(float)


def block_inverse_tpc(F, S, lams, lam, cs):
    """Six-face analogue of Alg. 1, batched over blocks (leading axis).

    F[d][s]: the residual on face s (s = 0, 1 at block position cs[s]) normal
    to x_(d+1); faces normal to x1 are indexed [i3, i2], normal to x2
    [i3, i1], normal to x3 [i2, i1].  The faces carry duplicated copies of
    their intersection lines; they are divided by their multiplicity first.
    S[d], lams[d]: 1D eigenvector matrices [i][k] and eigenvalues per block.
    Returns U[d][s] in the same layout.
    """
    nS = F[0][0].shape[-1]
    mult = face_multiplicity(nS, cs)
    F = [[F[d][s] / mult for s in range(2)] for d in range(3)]
    S1, S2, S3 = S
    l1, l2, l3 = lams
    T = np.swapaxes
    G = [[T(S3, 1, 2) @ F[0][s] @ S2 for s in range(2)],     # (k3, k2)
         [T(S3, 1, 2) @ F[1][s] @ S1 for s in range(2)],     # (k3, k1)
         [T(S2, 1, 2) @ F[2][s] @ S1 for s in range(2)]]     # (k2, k1)
    a = [[Sd[:, cs[s], :] for s in range(2)] for Sd in (S1, S2, S3)]
    E = 0.0
    for s in range(2):
        E = (E + a[0][s][:, None, None, :] * G[0][s][:, :, :, None]
             + a[1][s][:, None, :, None] * G[1][s][:, :, None, :]
             + a[2][s][:, :, None, None] * G[2][s][:, None, :, :])
    D = lam + l1[:, None, None, :] + l2[:, None, :, None] + l3[:, :, None, None]
    V = E / D
    U = [[None, None], [None, None], [None, None]]
    for s in range(2):
        H1 = np.einsum("zabk,zk->zab", V, a[0][s])
        H2 = np.einsum("zakb,zk->zab", V, a[1][s])
        H3 = np.einsum("zkab,zk->zab", V, a[2][s])
        U[0][s] = S3 @ H1 @ T(S2, 1, 2)
        U[1][s] = S3 @ H2 @ T(S1, 1, 2)
        U[2][s] = S2 @ H3 @ T(S1, 1, 2)
    return U


def block_inverse_tpf(F, S, lams, lam, cs):
    """Full-block fast diagonalization restricted to the six faces.

    The face residual (each node once) is placed in the full n_S^3 block,
    mapped by (S^T x S^T x S^T), scaled by the inverse eigenvalue sums and
    mapped back (eq. fast_diagonalization); the faces are then read off.
    """
    nS = F[0][0].shape[-1]
    nb = F[0][0].shape[0]
    R = np.zeros((nb, nS, nS, nS))          # [i3, i2, i1]
    on = np.zeros(nS, dtype=bool)
    on[list(cs)] = True
    for s in range(2):
        c = cs[s]
        R[:, :, :, c] = F[0][s]
        m2 = ~on[None, :] & np.ones((nS, 1), dtype=bool)        # i1 not on a face position
        R[:, :, c, :] = np.where(m2, F[1][s], R[:, :, c, :])
        m3 = ~on[:, None] & ~on[None, :]
        R[:, c, :, :] = np.where(m3, F[2][s], R[:, c, :, :])
    S1, S2, S3 = S
    l1, l2, l3 = lams
    T = np.swapaxes

    def ax1(A, u):
        return np.matmul(u, T(A, 1, 2)[:, None])

    def ax2(A, u):
        return np.matmul(A[:, None], u)

    def ax3(A, u):
        E_, n3, n2, n1 = u.shape
        return np.matmul(A, u.reshape(E_, n3, n2 * n1)).reshape(E_, A.shape[1], n2, n1)

    t = ax3(T(S3, 1, 2), ax2(T(S2, 1, 2), ax1(T(S1, 1, 2), R)))
    D = lam + l1[:, None, None, :] + l2[:, None, :, None] + l3[:, :, None, None]
    u = ax3(S3, ax2(S2, ax1(S1, t / D)))
    return [[u[:, :, :, cs[s]] for s in range(2)],
            [u[:, :, cs[s], :] for s in range(2)],
            [u[:, cs[s], :, :] for s in range(2)]]


class _Blocks:
    """Block index maps and gathered 1D tables for a mesh."""

    def __init__(self, mesh: Mesh, weights="smooth"):
        p = mesh.p
        nS = 3 * p - 1
        n1, n2, n3 = mesh.n
        N1, N2, N3 = mesh.N
        self.cs = (p - 1, 2 * p - 1)
        tabs = []
        for d in range(3):
            Ss, ls, ws = [], [], []
            for e in range(mesh.n[d]):
                S, lam, _ = block_tables_1d(mesh.h[d], p, e, mesh.bc[d])
                Ss.append(S)
                ls.append(lam)
                ws.append(block_weights_1d(mesh.n[d], p, e, weights, periodic=mesh.periodic[d]))
            tabs.append((np.array(Ss), np.array(ls), np.array(ws)))
        e3, e2, e1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
        e1, e2, e3 = e1.ravel(), e2.ravel(), e3.ravel()
        self.S = [tabs[0][0][e1], tabs[1][0][e2], tabs[2][0][e3]]
        self.l = [tabs[0][1][e1], tabs[1][1][e2], tabs[2][1][e3]]
        self.w = [tabs[0][2][e1], tabs[1][2][e2], tabs[2][2][e3]]
        sentinel = N1 * N2 * N3
        self.sentinel = sentinel

        def flat(i1, i2, i3):
            i1, i2, i3 = mesh.wrap(0, i1), mesh.wrap(1, i2), mesh.wrap(2, i3)
            ok = (i1 >= 0) & (i1 < N1) & (i2 >= 0) & (i2 < N2) & (i3 >= 0) & (i3 < N3)
            return np.where(ok, (i3 * N2 + i2) * N1 + i1, sentinel)

        o = np.arange(nS)
        b1, b2, b3 = (e1 - 1) * p + 1, (e2 - 1) * p + 1, (e3 - 1) * p + 1   # global index of position 0
        A = o[None, :, None]        # rows
        B = o[None, None, :]        # columns
        col = lambda x: x[:, None, None]
        self.idx = [[None, None], [None, None], [None, None]]
        for s in range(2):
            cpos = self.cs[s]
            # normal x1: [i3, i2]; normal x2: [i3, i1]; normal x3: [i2, i1]
            self.idx[0][s] = flat(col(b1) + cpos, col(b2) + B, col(b3) + A)
            self.idx[1][s] = flat(col(b1) + B, col(b2) + cpos, col(b3) + A)
            self.idx[2][s] = flat(col(b1) + B, col(b2) + A, col(b3) + cpos)
        # the 2D weight of a face position: product of the block's 1D weights
        self.W = [[None, None], [None, None], [None, None]]
        w1, w2, w3 = self.w
        for s in range(2):
            cpos = self.cs[s]
            self.W[0][s] = w1[:, cpos][:, None, None] * w3[:, :, None] * w2[:, None, :]
            self.W[1][s] = w2[:, cpos][:, None, None] * w3[:, :, None] * w1[:, None, :]
            self.W[2][s] = w3[:, cpos][:, None, None] * w2[:, :, None] * w1[:, None, :]
        # each node is added once: on the face of the lowest direction that contains it
        on = np.zeros(nS, dtype=bool)
        on[list(self.cs)] = True
        self.keep = [np.ones((nS, nS), dtype=bool),
                     np.broadcast_to(~on[None, :], (nS, nS)),
                     ~on[:, None] & ~on[None, :]]
        self.free = mesh.free_skeleton_mask().ravel()


def _blocks(mesh: Mesh, weights="smooth") -> _Blocks:
    key = "_oracle_blocks_" + weights
    cache = getattr(mesh, key, None)
    if cache is None:
        cache = _Blocks(mesh, weights)
        setattr(mesh, key, cache)
    return cache


def block_smoother(mesh: Mesh, r_grid, omega: float = 1.0, route: str = "tpc",
                   weights: str = "smooth", chunk: int = 512):
    """du = omega sum_e W_e R_e^T Hhat_e^-1 R_e r over all element-centred
    blocks (eq. smoother_definition with the blocks of Sec. 3.4)."""
    if mesh.p < 2:
        raise ValueError("element-centred blocks need p >= 2")
    bl = _blocks(mesh, weights)
    r = np.append(np.asarray(r_grid, dtype=np.float64).ravel(), 0.0)
    r = np.where(np.append(bl.free, False), r, 0.0)
    nb = bl.S[0].shape[0]
    N = bl.sentinel
    du = np.zeros(N + 1)
    inv = block_inverse_tpc if route == "tpc" else block_inverse_tpf
    for b0 in range(0, nb, chunk):
        sl = slice(b0, min(nb, b0 + chunk))
        F = [[r[bl.idx[d][s][sl]] for s in range(2)] for d in range(3)]
        U = inv(F, [x[sl] for x in bl.S], [x[sl] for x in bl.l], mesh.lam, bl.cs)
        for d in range(3):
            for s in range(2):
                ii = bl.idx[d][s][sl]
                vals = np.where(bl.keep[d][None], U[d][s] * bl.W[d][s][sl], 0.0)
                du += np.bincount(ii.ravel(), weights=vals.ravel(), minlength=N + 1)
    du = np.where(bl.free, du[:N], 0.0)
    return omega * du.reshape(mesh.shape)
