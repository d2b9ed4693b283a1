"""GPU parity of the exact coarse solve by fast diagonalization (FP64)
against the oracle's (oracle/coarse_fd.py, pinned to the dense
Schur-complement solve), in the coarse-solve entry point, in the V-cycle
and in whole solves, on meshes with ragged element counts, one element in a
direction, stretched widths and lambda = 0; and at full size on the p = 2
and p = 8 sweep points."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import bench
import paper_1808_03595_amd as pmg
import synth
from oracle import coarse_fd, matfree, solver
from tests.gpu_helpers import LevelIO, make_pair, rel

pytestmark = pytest.mark.gpu

CASES = [
    # (n, p, lambda, alpha): the bottom level is p_0 = 2 (p >= 3), or the
    # whole problem (p <= 2)
    ((5, 3, 4), 4, 1.0, 1.2),
    ((3, 1, 2), 6, 0.0, 1.0),
    ((7, 6, 5), 2, 1.0, 1.3),
    ((4, 5, 3), 1, 2.0, 1.0),
    ((2, 2, 2), 12, 1.0, 1.1),
]


def _cid(c):
    return f"n{c[0][0]}{c[0][1]}{c[0][2]}-p{c[1]}"


@pytest.mark.parametrize("case", CASES, ids=_cid)
def test_fd_coarse_solve(gpu, case):
    n, p, lam, alpha = case
    g, o = make_pair(n, p, lam, alpha)
    g.set_coarse_solver(1)
    io = LevelIO(g, 0)
    o0 = o.with_degree(io.p)
    for seed in (51, 52):
        b = synth.random_grid(o0.shape, seed) * o0.free_skeleton_mask()
        x = torch.full((io.len,), float("nan"), dtype=torch.float64, device=gpu)
        it = g.coarse_solve(io.to_dev(b), x)
        assert it == 0
        xx = x.cpu().numpy()
        assert np.isfinite(xx).all()
        assert not np.any(xx[np.setdiff1d(np.arange(io.len), io.slot)]), "slot without an unknown written"
        ref = coarse_fd.fd_condensed_solve(o0, b)
        assert rel(io.to_grid(x), ref) <= 1e-12
        # and it solves the condensed system: the oracle's residual
        r = b - matfree.condensed_op(o0, io.to_grid(x))
        assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(b)
    g.close()


@pytest.mark.parametrize("case", CASES[:2] + CASES[4:], ids=_cid)
def test_vcycle_with_fd_coarse(gpu, case):
    """Alg. 3 with the exact coarse solve: FP64 against the oracle's V-cycle
    with its fast-diagonalization coarse solve, FP32 at the FP32 bound."""
    n, p, lam, alpha = case
    g, o = make_pair(n, p, lam, alpha)
    g.set_coarse_solver(1)
    io = LevelIO(g, g.num_levels())
    r = synth.random_grid(o.shape, 53) * o.free_skeleton_mask()
    ref = solver.Hierarchy(o, coarse="fd").vcycle(None, r)
    z = torch.full((io.len,), float("nan"), dtype=torch.float64, device=gpu)
    g.vcycle(io.to_dev(r), z, pmg.F64)
    torch.cuda.synchronize()
    assert rel(io.to_grid(z), ref) <= 1e-11
    z32 = torch.full((io.len,), float("nan"), dtype=torch.float32, device=gpu)
    g.vcycle(io.to_dev(r / np.linalg.norm(r), torch.float32), z32, pmg.F32)
    torch.cuda.synchronize()
    assert rel(io.to_grid(z32) * np.linalg.norm(r), ref) <= 1e-4
    g.close()


@pytest.mark.parametrize("case", CASES, ids=_cid)
def test_pcg_with_fd_coarse(gpu, case):
    """ipCG (Alg. 5) with the exact coarse solve, FP64 and mixed, against the
    oracle's solve: iteration count within one, solution to 1e-9; with no
    smoothed level (p <= 2) the preconditioner is the exact inverse and one
    iteration suffices."""
    n, p, lam, alpha = case
    g, o = make_pair(n, p, lam, alpha)
    g.set_coarse_solver(1)
    f = synth.random_grid(o.shape, 54)
    ref = solver.solve(o, f, method="kMG", rtol=1e-10, coarse="fd")
    for dt in (pmg.F64, pmg.F32):
        u = torch.zeros(o.shape, dtype=torch.float64, device=gpu)
        st = g.pcg_solve(torch.as_tensor(f, device=gpu), u, 1e-10, 100, dt)
        assert st.status == 0 and st.rel_res <= 1e-10
        assert st.coarse_iters == 0
        assert abs(st.iters - ref.iters) <= 1, (dt, st.iters, ref.iters)
        if p <= 2:
            assert st.iters <= (1 if dt == pmg.F64 else 3)
        assert rel(u.cpu().numpy(), ref.u) <= 1e-9
    g.close()


def test_switch_between_coarse_solvers(gpu):
    """CG, exact, CG again on one handle: the solver graphs are rebuilt and
    every solve meets its tolerance; with the exact coarse solve the MG
    iteration (Alg. 4) needs no more iterations than with the CG."""
    g, o = make_pair((6, 5, 4), 8, 1.0, 1.2)
    g.set_cycle(0, 3e-2, 2000)
    f = torch.as_tensor(synth.random_grid(o.shape, 55), device=gpu)
    its = []
    for kind in (0, 1, 0):
        g.set_coarse_solver(kind)
        u = torch.zeros_like(f)
        st = g.pcg_solve(f, u, 1e-10, 100, pmg.F32)
        assert st.status == 0 and st.rel_res <= 1e-10
        u = torch.zeros_like(f)
        st2 = g.mg_solve(f, u, 1e-10, 100)
        assert st2.status == 0
        its.append(st2.iters)
    assert its[1] <= its[0] and its[2] == its[0]
    g.close()


@pytest.mark.parametrize("p", [2, 8])
def test_fd_coarse_full_size(gpu, p):
    """The p-sweep points p = 2 (108^3 elements: the exact solve is the whole
    condensed problem, 9.9M unknowns) and p = 8 (27^3 elements, levels
    2, 4, 8): the oracle's residual of the returned solution and its
    interior recovery."""
    wl = bench.workload(f"c3p{p}")
    g = bench.create(pmg, wl)
    g.set_coarse_solver(1)
    o = bench.oracle_mesh(wl)
    u_ex, f = bench.make_rhs(g, wl, torch, synth, gpu)
    f_h = f.cpu().numpy()
    F_hat = matfree.condense_rhs(o, f_h)
    mask = o.free_skeleton_mask()
    for dt in (pmg.F64, pmg.F32):
        u = torch.zeros_like(f)
        st = g.pcg_solve(f, u, 1e-10, 100, dt)
        assert st.status == 0 and st.rel_res <= 1e-10
        uh = u.cpu().numpy()
        r = F_hat - matfree.condensed_op(o, uh * mask)
        assert np.linalg.norm(r[mask]) <= 2e-10 * np.linalg.norm(F_hat[mask])
        assert rel(uh, matfree.recover_interior(o, f_h, uh * mask)) <= 1e-12
    g.close()


@pytest.mark.parametrize("case,level", [(((3, 2, 3), 8, 1.0, 1.2), 1), (((2, 3, 2), 12, 0.5, 1.0), 2),
                                        (((3, 3, 2), 16, 1.0, 1.1), 1)])
def test_coarse_level_above_zero(gpu, case, level):
    """Exact solve on p-level k > 0: the coarse solve of that level, the
    V-cycle (FP64 and FP32) and whole solves against the oracle's hierarchy
    with the same coarse level."""
    n, p, lam, alpha = case
    g, o = make_pair(n, p, lam, alpha)
    g.set_coarse_solver(1)
    g.set_coarse_level(level)
    ioc = LevelIO(g, level)
    oc = o.with_degree(ioc.p)
    b = synth.random_grid(oc.shape, 61) * oc.free_skeleton_mask()
    x = torch.full((ioc.len,), float("nan"), dtype=torch.float64, device=gpu)
    assert g.coarse_solve(ioc.to_dev(b), x) == 0
    assert rel(ioc.to_grid(x), coarse_fd.fd_condensed_solve(oc, b)) <= 1e-12
    io = LevelIO(g, g.num_levels())
    r = synth.random_grid(o.shape, 62) * o.free_skeleton_mask()
    ref = solver.Hierarchy(o, coarse="fd", coarse_level=level).vcycle(None, r)
    z = torch.full((io.len,), float("nan"), dtype=torch.float64, device=gpu)
    g.vcycle(io.to_dev(r), z, pmg.F64)
    torch.cuda.synchronize()
    assert rel(io.to_grid(z), ref) <= 1e-11
    z32 = torch.full((io.len,), float("nan"), dtype=torch.float32, device=gpu)
    g.vcycle(io.to_dev(r / np.linalg.norm(r), torch.float32), z32, pmg.F32)
    torch.cuda.synchronize()
    assert rel(io.to_grid(z32) * np.linalg.norm(r), ref) <= 1e-4
    f = synth.random_grid(o.shape, 63)
    sref = solver.solve(o, f, method="kMG", rtol=1e-10, coarse="fd", coarse_level=level)
    for dt in (pmg.F64, pmg.F32):
        u = torch.zeros(o.shape, dtype=torch.float64, device=gpu)
        st = g.pcg_solve(torch.as_tensor(f, device=gpu), u, 1e-10, 100, dt)
        assert st.status == 0 and st.rel_res <= 1e-10
        assert abs(st.iters - sref.iters) <= 1, (dt, st.iters, sref.iters)
        assert rel(u.cpu().numpy(), sref.u) <= 1e-9
    # back to level 0: the default cycle again
    g.set_coarse_level(0)
    u = torch.zeros(o.shape, dtype=torch.float64, device=gpu)
    st = g.pcg_solve(torch.as_tensor(f, device=gpu), u, 1e-10, 100, pmg.F64)
    assert st.status == 0
    assert abs(st.iters - solver.solve(o, f, rtol=1e-10, coarse="fd").iters) <= 1
    g.close()


def test_coarse_level_refusals(gpu):
    g, o = make_pair((3, 2, 3), 8, 1.0, 1.0)
    g.set_coarse_solver(0)
    with pytest.raises(pmg.PmgError) as ei:
        g.set_coarse_level(1)                 # the coarse CG runs on level 0
    assert ei.value.code == pmg.EUNSUP
    g.set_coarse_solver(1)
    g.set_coarse_level(1)
    with pytest.raises(pmg.PmgError) as ei:
        g.set_coarse_solver(0)
    assert ei.value.code == pmg.EUNSUP
    with pytest.raises(pmg.PmgError) as ei:
        g.set_coarse_level(3)                 # levels 0..2
    assert ei.value.code == pmg.EINVAL
    g.close()
