"""Shared helpers of the GPU tests: device arrays and oracle grids."""
from __future__ import annotations

import numpy as np
import torch

import paper_1808_03595_amd as pmg
from oracle import mesh as omesh


def make_pair(n, p, lam, alpha=1.0, widths=None, bc=None):
    """Build the GPU mesh and the oracle mesh of the same problem (boundary
    kinds ``bc`` as the oracle's mesh takes them; Dirichlet if None)."""
    if bc is not None:
        o = omesh.Mesh.box(n, p, lam, alpha, bc=bc) if widths is None else \
            omesh.Mesh(widths[0], widths[1], widths[2], p, lam, bc)
        g = pmg.create_mesh_bc(o.h[0], o.h[1], o.h[2], p, lam, o.bc)
        return g, o
    if widths is None:
        g = pmg.create_mesh(n[0], n[1], n[2], p, lam, alpha)
        o = omesh.Mesh.box(n, p, lam, alpha)
    else:
        g = pmg.create_mesh_widths(widths[0], widths[1], widths[2], p, lam)
        o = omesh.Mesh(widths[0], widths[1], widths[2], p, lam)
    return g, o


def level_mesh(o, g, level):
    return o.with_degree(g.level_degree(level))


def to_skel(g, grid, level=None, dtype=torch.float64):
    """Oracle grid (finest level only) -> GPU skeleton array via the HIP path."""
    dev = torch.device("cuda:0")
    gd = torch.as_tensor(np.ascontiguousarray(grid), dtype=torch.float64, device=dev)
    s = torch.empty(g.skeleton_len(), dtype=dtype, device=dev)
    g.grid_to_skeleton(gd, s, pmg.F64 if dtype == torch.float64 else pmg.F32)
    return s


def from_skel(g, s):
    dev = torch.device("cuda:0")
    out = torch.empty(g.grid_shape(), dtype=torch.float64, device=dev)
    g.skeleton_to_grid(s, out, pmg.F64 if s.dtype == torch.float64 else pmg.F32)
    torch.cuda.synchronize()
    return out.cpu().numpy()


class LevelIO:
    """Grid <-> skeleton conversion on any level, done on the host.

    The HIP library only converts on the finest level; coarser levels are
    filled here by the plain storage rule of the plane layout (each unknown
    once: i1 % p == 0 -> family 0, else i2 % p == 0 -> family 1, else
    family 2), which the finest-level round trip pins.
    """

    def __init__(self, g, level, bc=None):
        self.g = g
        self.p = g.level_degree(level)
        n = g.n
        self.len = g.skeleton_len(level)
        p = self.p
        N = [n[d] * p + 1 for d in range(3)]
        pad = lambda v: (v + 3) & ~3
        pitch = [pad(N[1]), pad(N[0]), pad(N[0])]
        rows = [N[2], N[2], N[1]]
        pst = [((rows[d] * pitch[d] + 63) // 64) * 64 for d in range(3)]
        off = [0, (n[0] + 1) * pst[0], (n[0] + 1) * pst[0] + (n[1] + 1) * pst[1]]
        assert off[2] + (n[2] + 1) * pst[2] == self.len
        i3, i2, i1 = np.meshgrid(np.arange(N[2]), np.arange(N[1]), np.arange(N[0]), indexing="ij")
        on1, on2, on3 = i1 % p == 0, i2 % p == 0, i3 % p == 0
        kinds = omesh.parse_bc(bc)
        ii = (i1, i2, i3)
        dirichlet = np.zeros(i1.shape, dtype=bool)
        for d in range(3):
            lo, hi = kinds[d]
            if lo == "D":
                dirichlet |= ii[d] == 0
            if hi == "D":
                dirichlet |= ii[d] == N[d] - 1
            if lo == "P":             # mirror layer: no unknown of its own
                dirichlet |= ii[d] == N[d] - 1
        skel = (on1 | on2 | on3) & ~dirichlet
        slot = np.where(on1, off[0] + (i1 // p) * pst[0] + i3 * pitch[0] + i2,
                        np.where(on2, off[1] + (i2 // p) * pst[1] + i3 * pitch[1] + i1,
                                 off[2] + (i3 // p) * pst[2] + i2 * pitch[2] + i1))
        self.mask = skel
        self.slot = slot[skel]
        self.shape = (N[2], N[1], N[0])

    def to_dev(self, grid, dtype=torch.float64):
        v = np.zeros(self.len)
        v[self.slot] = np.asarray(grid)[self.mask]
        return torch.as_tensor(v, dtype=dtype, device="cuda:0")

    def to_grid(self, s):
        v = s.detach().double().cpu().numpy()
        out = np.zeros(self.shape)
        out[self.mask] = v[self.slot]
        return out


def rel(a, b):
    """Relative difference of a from the reference b that every parity check
    compares with its tolerance tol: the larger of the norm-wise difference
    ||a - b||_2 / ||b||_2 and one fifth of the largest element difference
    relative to the largest reference magnitude, max|a - b| / (5 max|b|).
    So `rel(a, b) <= tol` also bounds every single element,
    max|a - b| <= 5 tol max|b|: one wrong entry of a long vector cannot hide
    in the norm."""
    a = np.ravel(np.asarray(a, dtype=np.float64))
    b = np.ravel(np.asarray(b, dtype=np.float64))
    d = a - b
    nb = np.linalg.norm(b)
    mb = np.max(np.abs(b)) if b.size else 0.0
    norm_wise = np.linalg.norm(d) / (nb if nb > 0 else 1.0)
    if not d.size:
        return norm_wise
    elem = np.max(np.abs(d)) / (5.0 * (mb if mb > 0 else 1.0))
    return max(norm_wise, elem)
