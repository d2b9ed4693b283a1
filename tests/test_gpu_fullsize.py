"""GPU parity at the full benchmark sizes, in the launch configuration that
bench.py times.

At these sizes the FP64 oracle still evaluates the condensed operator, the
star smoother, condensation and recovery over whole vectors in seconds, so
those outputs are compared element by element (same bars as the small
cases: 1e-12 relative in FP64, the FP32 bound of the small cases).  Whole
solves are checked by properties that hold at any size: the residual of
the returned solution recomputed by the oracle (F_hat - H_hat u_hat, Sec. 2.2)
must be below the solver's tolerance, the interior must be the oracle's
recovery of the returned skeleton values (Alg. 4, last step), and the error
against the manufactured solution must be at the discretisation level.

Workloads: 16^3 elements at p = 8 and 8^3 at p = 16, geometrically stretched
to aspect ratio 8 (the benchmark's main workload and its p = 16 twin);
4^3 elements at p = 48 (the largest degree of the p sweep); 32^3 elements at
p = 8 on anisotropic boxes (0, AR) x (0, ceil(AR / 2) / 2) x (0, 1) with
lambda in {0, 1e2, 1e4} for the mixed-precision solver.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import bench
import paper_1808_03595_amd as pmg
import synth
from oracle import matfree
from oracle import mesh as omesh
from tests.gpu_helpers import LevelIO, make_pair, rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5

OPERATOR_CASES = [
    # (n, p, lambda, alpha)
    ((16, 16, 16), 8, 1.0, 8.0 ** (1.0 / 15.0)),
    ((8, 8, 8), 16, 1.0, 8.0 ** (1.0 / 7.0)),
    ((4, 4, 4), 48, 1.0, 1.0),
]


def _oid(c):
    return f"n{c[0][0]}-p{c[1]}"


@pytest.mark.parametrize("case", OPERATOR_CASES, ids=_oid)
def test_operator_and_smoother_full_size(gpu, case):
    n, p, lam, alpha = case
    g, o = make_pair(n, p, lam, alpha)
    for level in range(g.num_levels() + 1):
        io = LevelIO(g, level)
        ol = o.with_degree(io.p)
        mask = ol.free_skeleton_mask()
        u = synth.random_grid(ol.shape, 101 + level) * mask
        ref_op = matfree.condensed_op(ol, u)
        ref_sm = matfree.smoother(ol, u, 0.9) if io.p >= 2 else None
        for dt, tdt, tol in ((pmg.F64, torch.float64, TOL64), (pmg.F32, torch.float32, TOL32)):
            du = io.to_dev(u, tdt)
            y = torch.full_like(du, float("nan"))
            g.apply_condensed_op(level, du, y, dt)
            torch.cuda.synchronize()
            err = rel(io.to_grid(y), ref_op)
            assert err <= tol, ("operator", level, dt, err)
            if ref_sm is not None:
                z = torch.full_like(du, float("nan"))
                g.schwarz_smooth(level, du, z, 0.9, dt)
                torch.cuda.synchronize()
                err = rel(io.to_grid(z), ref_sm)
                assert err <= tol, ("smoother", level, dt, err)
    g.close()


def test_degree2_operator_and_smoother_large(gpu):
    """p = 2 on 81 x 80 x 82 elements (551k stars): the smoother runs as
    eight launches of stars with disjoint windows and plain adds (taken from
    2^19 stars on), the operator as the per-node axis stencil; both against
    the oracle over whole vectors."""
    g, o = make_pair((81, 80, 82), 2, 1.0, 1.01)
    io = LevelIO(g, 0)
    mask = o.free_skeleton_mask()
    u = synth.random_grid(o.shape, 23) * mask
    ref_op = matfree.condensed_op(o, u)
    ref_sm = matfree.smoother(o, u, 0.7)
    for dt, tdt, tol in ((pmg.F64, torch.float64, TOL64), (pmg.F32, torch.float32, TOL32)):
        du = io.to_dev(u, tdt)
        y = torch.full_like(du, float("nan"))
        g.apply_condensed_op(0, du, y, dt)
        z = torch.full_like(du, float("nan"))
        g.schwarz_smooth(0, du, z, 0.7, dt)
        torch.cuda.synchronize()
        assert rel(io.to_grid(y), ref_op) <= tol, dt
        assert rel(io.to_grid(z), ref_sm) <= tol, dt
    g.close()


def _check_solution(o, f, u, F_hat, tol_res):
    """Residual of the returned skeleton values and consistency of the
    interior, both recomputed by the oracle."""
    mask = o.free_skeleton_mask()
    u_hat = u * mask
    r = F_hat - matfree.condensed_op(o, u_hat)
    res = np.linalg.norm(r[mask]) / np.linalg.norm(F_hat[mask])
    assert res <= tol_res, res
    rec = matfree.recover_interior(o, f, u_hat)
    assert rel(u, rec) <= 1e-12
    return res


def test_benchmark_workload_solves(gpu):
    """16^3 elements, p = 8, stretched to AR 8, lambda = 1, 8 sine modes: the
    benchmark's three solvers (FP64; FP32 cycle with omega = 1; FP32 cycle
    with the learned damping), as bench.py runs them."""
    wl = bench.workload("c2a")
    n, p = wl["n"], wl["p"]
    g, o = make_pair(n, p, wl["lam"], wl["alpha"])
    g.set_cycle(0, 3e-2, 2000)
    u_ex, f = bench.make_rhs(g, wl, torch, synth, gpu)
    f_h = f.cpu().numpy()
    u_ex_h = u_ex.cpu().numpy()
    F_hat = matfree.condense_rhs(o, f_h)
    omega = bench.learned_damping(wl, g.num_levels())
    for dtype, om in ((pmg.F64, None), (pmg.F32, None), (pmg.F32, omega)):
        g.set_damping(om)
        u = torch.zeros_like(f)
        st = g.pcg_solve(f, u, 1e-10, 200, dtype)
        assert st.status == 0 and st.rel_res <= 1e-10
        uh = u.cpu().numpy()
        _check_solution(o, f_h, uh, F_hat, 2e-10)
        assert rel(uh, u_ex_h) <= 1e-9
    g.close()


@pytest.mark.parametrize("ar,lam", [(16, 1e4), (16, 0.0), (8, 1e2), (4, 1e2), (2, 0.0), (1, 0.0)])
def test_mixed_precision_32cubed(gpu, ar, lam):
    """32^3 elements, p = 8 (16.8M unknowns) on the anisotropic box: the FP32
    cycle inside FP64 CG reaches 1e-10, its solution agrees with the FP64
    solver's, and the oracle's residual of it is below the tolerance."""
    n, p = (32, 32, 32), 8
    lengths = (float(ar), math.ceil(ar / 2) / 2.0, 1.0)
    widths = [np.full(n[d], lengths[d] / n[d]) for d in range(3)]
    g, o = make_pair(n, p, lam, widths=widths)
    g.set_cycle(0, 3e-2, 2000)
    X3, X2, X1 = o.coords()
    k, a = synth.sine_modes(3)
    u_ex, f = synth.sine_solution(k, a, lengths, X1, X2, X3, lam)
    f = np.broadcast_to(f, o.shape).copy()
    u_ex = np.broadcast_to(u_ex, o.shape).copy()
    df = torch.as_tensor(f, device=gpu)
    sols = {}
    for dtype in (pmg.F64, pmg.F32):
        u = torch.zeros_like(df)
        st = g.pcg_solve(df, u, 1e-10, 300, dtype)
        assert st.status == 0 and st.rel_res <= 1e-10, (dtype, st.status, st.rel_res)
        sols[dtype] = u.cpu().numpy()
    F_hat = matfree.condense_rhs(o, f)
    _check_solution(o, f, sols[pmg.F32], F_hat, 2e-10)
    assert rel(sols[pmg.F32], sols[pmg.F64]) <= 1e-8
    assert rel(sols[pmg.F32], u_ex) <= 1e-6
    g.close()
