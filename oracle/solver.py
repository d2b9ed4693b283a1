"""p-multigrid V-cycle and the outer solvers (oracle, FP64).

Passages followed:
* Sec. 4.1, level degrees p_l = p_0 2^l (l < L), p_L = p, p_0 = 2;
  Alg. 3 (V-cycle) with nu_pre,l = nu_post,l = 1 ("kMG") or 2^(L-l)
  ("kvMG"); coarse-grid CG on the condensed system at p_0 = 2;
* Alg. 4 (MG solver: V-cycles as a fixed-point iteration);
* Alg. 5 (Krylov-accelerated MG: inexact preconditioned CG with the
  V-cycle as preconditioner);
* Sec. 5.2, convergence rate rho = (|r_n10| / |r_0|)^(1/n10).

Readings where the paper is silent (each also listed in the design notes):
* the coarse CG is Jacobi-preconditioned (diagonal of the condensed
  operator) and stops when the D^-1-weighted residual norm has dropped by
  ``coarse_rtol`` or after ``coarse_maxit`` iterations; ``coarse_rtol = 0``
  gives a fixed iteration count;
* the per-level damping omega_l multiplies the smoother output
  (u_l += omega_l Smoother(...)); omega_l = 1 is the paper's method;
  ``omega[j]`` is indexed from the finest level (j = L - l);
* stopping test |r|_2 <= rtol |r_0|_2 over the unique condensed unknowns.

Optional extension below p_0 (``hmg_levels`` > 0; not the paper's coarse
solver, but the remedy its complexity discussion (Sec. 4.2) names for the
O(n_e^(4/3)) coarse cost: a low-order multigrid): the p_0 = 2 level is
followed by degree-1 levels, first on the same mesh (p-transfer 2 -> 1), then
on meshes with pairs of elements merged in every direction (trilinear
h-transfers), each smoothed by the star smoother of degree 1 (a damped
point-Jacobi step, damping ``hmg_omega``) with ``hmg_nu`` pre- and
post-smoothing steps; the coarse CG then runs on the smallest mesh.
"""
from __future__ import annotations

import numpy as np

from . import blocks, coarse_fd, matfree
from .mesh import Mesh, level_degrees


def dot(a, b):
    return float(np.sum(np.asarray(a) * np.asarray(b)))


def norm(a):
    return float(np.sqrt(dot(a, a)))


class Hierarchy:
    """Levels 0..L of one mesh and the V-cycle of Alg. 3."""

    def __init__(self, mesh: Mesh, nu_mode: str = "kMG", omega=None,
                 coarse_rtol: float = 1e-8, coarse_maxit: int = 2000,
                 exact_coarse: bool = False, hmg_levels: int = 0,
                 hmg_omega: float = 0.6, hmg_nu: int = 1,
                 smoother: str = "star", block_weights: str = "smooth", coarse: str = "cg",
                 coarse_level: int = 0):
        # coarse_level k > 0: the exact coarse solve inverts the condensed
        # system of p-level k; the levels below it are not part of the cycle
        self.degs = level_degrees(mesh.p)
        if coarse_level:
            if coarse != "fd" and not exact_coarse:
                raise ValueError("a coarse level above 0 needs an exact coarse solve")
            if hmg_levels:
                raise ValueError("a coarse level above 0 excludes degree-1 levels")
            if not 0 < coarse_level < len(self.degs):
                raise ValueError("coarse level out of range")
            self.degs = self.degs[coarse_level:]
        Lp = len(self.degs) - 1
        pmeshes = [mesh.with_degree(q) for q in self.degs]
        pmeshes[-1] = mesh
        # levels below p_0: degree 1 on the same mesh, then merged meshes
        hmeshes = []
        if hmg_levels > 0 and self.degs[0] >= 2:
            if not mesh.all_dirichlet():
                raise NotImplementedError("degree-1 h-levels: Dirichlet boundaries only")
            cur = mesh.with_degree(1)
            hmeshes.append(cur)
            for _ in range(hmg_levels - 1):
                if any(len(h) % 2 or len(h) < 4 for h in cur.h):
                    break
                cur = Mesh(*(matfree.merged_widths(h) for h in cur.h), 1, mesh.lam)
                hmeshes.append(cur)
        self.nh = len(hmeshes)
        self.meshes = hmeshes[::-1] + pmeshes
        self.L = L = len(self.meshes) - 1
        # transfer kind between level l-1 and l: "h" (merged mesh) or "p"
        self.kind = [None] + ["h" if self.meshes[l].n != self.meshes[l - 1].n else "p"
                              for l in range(1, L + 1)]
        nh = self.nh
        if nu_mode == "kMG":
            self.nu = [1] * (L + 1)
        elif nu_mode == "kvMG":
            self.nu = [2 ** (L - l) for l in range(L + 1)]
        else:
            raise ValueError(nu_mode)
        for l in range(nh + 1):          # degree-1 levels and the old p_0 level
            if l < nh:
                self.nu[l] = hmg_nu
        if nu_mode == "kvMG":
            for l in range(nh, L + 1):
                self.nu[l] = 2 ** (L - l)
        om = [1.0] * (L + 1)
        for l in range(nh):
            om[l] = hmg_omega
        if omega is not None:
            for j, w in enumerate(omega):
                if j <= Lp - 1:
                    om[L - j] = float(w)
        self.omega = om
        self.coarse_rtol = coarse_rtol
        self.coarse_maxit = coarse_maxit
        self.exact_coarse = exact_coarse
        self._diag0 = None
        self._dense0 = None
        self.coarse_iters = []
        if smoother not in ("star", "element"):
            raise ValueError(smoother)
        self.smoother = smoother
        self.block_weights = block_weights
        if coarse not in ("cg", "fd"):
            raise ValueError(coarse)
        self.coarse = coarse

    def _prolong(self, l, uc):
        if self.kind[l] == "h":
            return matfree.h_prolong(self.meshes[l - 1], self.meshes[l], uc)
        return matfree.prolong(self.meshes[l - 1], self.meshes[l], uc)

    def _restrict(self, l, rf):
        if self.kind[l] == "h":
            return matfree.h_restrict(self.meshes[l], self.meshes[l - 1], rf)
        return matfree.restrict(self.meshes[l], self.meshes[l - 1], rf)

    # ---- coarse grid ----------------------------------------------------
    def coarse_solve(self, F0):
        m0 = self.meshes[0]
        if self.coarse == "fd":
            return coarse_fd.fd_condensed_solve(m0, F0)
        if self.exact_coarse:
            if self._dense0 is None:
                from .dense import CondensedSystem
                self._dense0 = CondensedSystem(m0)
            cs = self._dense0
            return cs.to_grid(np.linalg.solve(cs.Hhat, cs.to_vec(F0)))
        if self._diag0 is None:
            self._diag0 = matfree.condensed_diagonal(m0)
        return jacobi_pcg(lambda x: matfree.condensed_op(m0, x), F0,
                          self._diag0, self.coarse_rtol, self.coarse_maxit,
                          self.coarse_iters)

    # ---- Alg. 3 -----------------------------------------------------------
    def vcycle(self, u, F):
        L = self.L
        ms = self.meshes
        us = [None] * (L + 1)
        Fs = [None] * (L + 1)
        us[L] = None if u is None else np.asarray(u, dtype=np.float64)
        Fs[L] = np.asarray(F, dtype=np.float64)

        def residual(l):
            if us[l] is None:
                return Fs[l]
            return Fs[l] - matfree.condensed_op(ms[l], us[l])

        def smooth(l):
            if self.smoother == "element" and ms[l].p >= 2:
                du = blocks.block_smoother(ms[l], residual(l), self.omega[l],
                                           weights=self.block_weights)
            else:
                du = matfree.smoother(ms[l], residual(l), self.omega[l])
            us[l] = du if us[l] is None else us[l] + du

        for l in range(L, 0, -1):
            if l != L:
                us[l] = None                       # u_l <- 0
            for _ in range(self.nu[l]):
                smooth(l)
            Fs[l - 1] = self._restrict(l, residual(l))
        us[0] = self.coarse_solve(Fs[0])
        for l in range(1, L + 1):
            pu = self._prolong(l, us[l - 1])
            us[l] = pu if us[l] is None else us[l] + pu
            for _ in range(self.nu[l]):
                smooth(l)
        return us[L]


def jacobi_pcg(apply, b, diag, rtol, maxit, log=None):
    """Jacobi-preconditioned conjugate gradients from x = 0 (textbook form).

    Per iteration: q = A p, alpha = (r, z) / (p, q), x += alpha p,
    r -= alpha q, z = D^-1 r, beta = (r, z)_new / (r, z)_old,
    p = z + beta p.  Stops when (r, D^-1 r) <= rtol^2 (b, D^-1 b) or after
    ``maxit`` updates of x.
    """
    x = np.zeros_like(b)
    r = np.array(b, dtype=np.float64)
    z = r / diag
    rz = dot(r, z)
    rz0 = rz
    p = z.copy()
    it = 0
    while rz > 0.0 and it < maxit:
        q = apply(p)
        alpha = rz / dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        z = r / diag
        rz_new = dot(r, z)
        if rz_new <= (rtol * rtol) * rz0:
            break
        p = z + (rz_new / rz) * p
        rz = rz_new
    if log is not None:
        log.append(it)
    return x


class SolveResult:
    def __init__(self, u, uhat, iters, hist):
        self.u = u
        self.uhat = uhat
        self.iters = iters
        self.hist = hist

    @property
    def rho(self):
        """Mean convergence rate over the iterations (Sec. 5.2)."""
        if self.iters == 0:
            return 0.0
        return (self.hist[-1] / self.hist[0]) ** (1.0 / self.iters)


def ipcg(mesh: Mesh, Fhat, rtol=1e-10, maxit=200, hier: Hierarchy = None,
         precond=None, **hkw):
    """Alg. 5 on the condensed system; returns (uhat, iters, history)."""
    hier = hier or Hierarchy(mesh, **hkw)
    A = lambda x: matfree.condensed_op(mesh, x)
    M = precond or (lambda r: hier.vcycle(None, r))
    u = np.zeros_like(Fhat)
    r = np.array(Fhat, dtype=np.float64)     # r = F - H u with u = 0
    s = r.copy()
    p = np.zeros_like(r)
    delta = 1.0
    hist = [norm(r)]
    eps = rtol * hist[0]
    it = 0
    while hist[-1] > eps and it < maxit:
        z = M(r)
        gamma = dot(z, r)
        gamma0 = dot(z, s)
        beta = (gamma - gamma0) / delta
        delta = gamma
        p = beta * p + z
        q = A(p)
        alpha = gamma / dot(q, p)
        s = r
        u = u + alpha * p
        r = r - alpha * q
        hist.append(norm(r))
        it += 1
    return u, it, hist


def mg_solve(mesh: Mesh, Fhat, rtol=1e-10, maxit=200, hier=None, **hkw):
    """Alg. 4: repeated V-cycles until |F - H u| <= rtol |F|."""
    hier = hier or Hierarchy(mesh, **hkw)
    u = np.zeros_like(Fhat)
    r = np.array(Fhat, dtype=np.float64)
    hist = [norm(r)]
    eps = rtol * hist[0]
    it = 0
    while hist[-1] > eps and it < maxit:
        u = hier.vcycle(u, Fhat)
        r = Fhat - matfree.condensed_op(mesh, u)
        hist.append(norm(r))
        it += 1
    return u, it, hist


def solve(mesh: Mesh, f_grid, method="kMG", rtol=1e-10, maxit=200, **hkw):
    """Full solve: condense, iterate, recover (Alg. 4 / Alg. 5)."""
    Fhat = matfree.condense_rhs(mesh, f_grid)
    if method == "MG":
        uhat, it, hist = mg_solve(mesh, Fhat, rtol, maxit, **hkw)
    else:
        nu_mode = "kvMG" if method == "kvMG" else "kMG"
        uhat, it, hist = ipcg(mesh, Fhat, rtol, maxit, nu_mode=nu_mode, **hkw)
    u = matfree.recover_interior(mesh, f_grid, uhat)
    return SolveResult(u, uhat, it, hist)
