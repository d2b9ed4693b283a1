"""GPU parity on meshes with Neumann and periodic sides (Sec. 3.3) against
the oracle (pinned in tests/test_oracle_bc.py).

Every kernel family meets a boundary of each kind: the operator (per-node
stencils at p <= 2, one wavefront per element at 3 <= p <= 16, the batched
launches beyond), the star smoothers (small, matrix-core, batched), the
transfers, condensation and recovery, the exact coarse solve and whole
solves.  Bars as in the Dirichlet parity tests: FP64 1e-12, FP32 2e-5,
both also bounding the largest element error.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_1808_03595_amd as pmg
import synth
from oracle import coarse_fd, matfree, solver
from tests.gpu_helpers import LevelIO, make_pair, rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5

# (n, p, lambda, alpha, bc)
CASES = [
    ((3, 2, 4), 1, 1.0, 1.2, ("P", "N", ("D", "N"))),
    ((4, 3, 3), 2, 0.5, 1.0, (("N", "D"), "P", "P")),
    ((3, 2, 2), 3, 1.0, 1.3, ("N", "N", "N")),
    ((3, 3, 2), 4, 0.0, 1.0, ("P", ("D", "N"), "N")),
    ((2, 3, 3), 6, 2.0, 1.25, (("N", "D"), "P", ("D", "N"))),
    ((3, 2, 3), 8, 1.0, 1.0, ("P", "D", "P")),
    ((3, 3, 3), 8, 1.0, 1.15, ("P", "P", "P")),
    ((3, 2, 2), 12, 1.0, 1.0, ("P", "N", ("N", "D"))),
    ((3, 1, 2), 24, 5.0, 1.0, ("P", ("D", "N"), "N")),
]


def _ids(c):
    bc = "".join(b if isinstance(b, str) else "".join(b) for b in c[4])
    return f"n{''.join(map(str, c[0]))}-p{c[1]}-{bc}"


def _pair(case):
    n, p, lam, alpha, bc = case
    return make_pair(n, p, lam, alpha, bc=bc)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_layout_roundtrip_with_seams(gpu, case):
    """grid -> skeleton keeps the unknowns (mirror and Dirichlet slots 0);
    skeleton -> grid writes a mirror node as a copy of the node it repeats."""
    g, o = _pair(case)
    io = LevelIO(g, g.num_levels(), o.bc)
    f = synth.random_grid(o.shape, 1)
    s = torch.empty(g.skeleton_len(), dtype=torch.float64, device=gpu)
    g.grid_to_skeleton(torch.as_tensor(f, device=gpu), s)
    u = f * o.free_skeleton_mask()
    assert torch.equal(s, io.to_dev(u))
    back = torch.empty(o.shape, dtype=torch.float64, device=gpu)
    g.skeleton_to_grid(s, back)
    assert np.array_equal(back.cpu().numpy(), o.expand_periodic(u))
    g.close()


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_and_smoother_all_levels(gpu, case, dtype):
    g, o = _pair(case)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    dt = pmg.F64 if dtype == "f64" else pmg.F32
    tol = TOL64 if dtype == "f64" else TOL32
    for level in range(g.num_levels() + 1):
        io = LevelIO(g, level, o.bc)
        ol = o.with_degree(io.p)
        u = synth.random_grid(ol.shape, 2 + level) * ol.free_skeleton_mask()
        du = io.to_dev(u, tdt)
        y = torch.full_like(du, float("nan"))
        g.apply_condensed_op(level, du, y, dt)
        torch.cuda.synchronize()
        assert not torch.isnan(y).any()
        assert rel(io.to_grid(y), matfree.condensed_op(ol, u)) <= tol, ("op", level)
        # the input's mirror slots are left cleared
        assert torch.equal(du, io.to_dev(u, tdt))
        # every slot that is not an unknown is 0
        assert float(y.double().abs().sum()) == pytest.approx(float(np.abs(io.to_grid(y)).sum()), rel=1e-12)
        r = synth.random_grid(ol.shape, 7 + level) * ol.free_skeleton_mask()
        z = torch.full_like(du, float("nan"))
        g.schwarz_smooth(level, io.to_dev(r, tdt), z, 0.8, dt)
        torch.cuda.synchronize()
        assert rel(io.to_grid(z), matfree.smoother(ol, r, 0.8)) <= tol, ("smoother", level)
        assert float(z.double().abs().sum()) == pytest.approx(float(np.abs(io.to_grid(z)).sum()), rel=1e-12)
    g.close()


@pytest.mark.parametrize("case", [c for c in CASES if c[1] >= 3], ids=_ids)
def test_transfers_with_seams(gpu, case):
    g, o = _pair(case)
    for level in range(1, g.num_levels() + 1):
        iof, ioc = LevelIO(g, level, o.bc), LevelIO(g, level - 1, o.bc)
        of, oc = o.with_degree(iof.p), o.with_degree(ioc.p)
        uc = synth.random_grid(oc.shape, 11) * oc.free_skeleton_mask()
        uf = synth.random_grid(of.shape, 12) * of.free_skeleton_mask()
        ref_p = uf + matfree.prolong(oc, of, uc)
        ref_r = matfree.restrict(of, oc, uf)
        for dt, tol in ((pmg.F64, TOL64), (pmg.F32, TOL32)):
            tdt = torch.float64 if dt == pmg.F64 else torch.float32
            dfine = iof.to_dev(uf, tdt)
            dc = ioc.to_dev(uc, tdt)
            g.prolong_add(level, dc, dfine, dt)
            dco = torch.full((ioc.len,), float("nan"), dtype=tdt, device=gpu)
            g.restrict(level, iof.to_dev(uf, tdt), dco, dt)
            torch.cuda.synchronize()
            assert rel(iof.to_grid(dfine), ref_p) <= tol
            assert rel(ioc.to_grid(dco), ref_r) <= tol
            assert torch.equal(dc, ioc.to_dev(uc, tdt))      # mirror slots cleared again
            assert float(dfine.double().abs().sum()) == pytest.approx(float(np.abs(iof.to_grid(dfine)).sum()), rel=1e-12)
            assert float(dco.double().abs().sum()) == pytest.approx(float(np.abs(ioc.to_grid(dco)).sum()), rel=1e-12)
    g.close()


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_condense_recover_and_coarse_solve(gpu, case):
    g, o = _pair(case)
    io = LevelIO(g, g.num_levels(), o.bc)
    # the right-hand side's mirror layer holds other values: it is ignored
    f = synth.random_grid(o.shape, 21)
    fp = o.expand_periodic(f)
    df = torch.as_tensor(f, device=gpu)
    Fh = torch.full((io.len,), float("nan"), dtype=torch.float64, device=gpu)
    g.condense_rhs(df, Fh)
    torch.cuda.synchronize()
    assert rel(io.to_grid(Fh), matfree.condense_rhs(o, fp)) <= TOL64
    uh = synth.random_grid(o.shape, 22) * o.free_skeleton_mask()
    ref_u = matfree.recover_interior(o, fp, uh)
    du = torch.full(o.shape, float("nan"), dtype=torch.float64, device=gpu)
    duh = io.to_dev(uh)
    g.recover_interior(df, duh, du)
    torch.cuda.synchronize()
    assert rel(du.cpu().numpy(), ref_u) <= TOL64
    assert torch.equal(duh, io.to_dev(uh))
    # exact coarse solve on level 0
    io0 = LevelIO(g, 0, o.bc)
    o0 = o.with_degree(io0.p)
    b = synth.random_grid(o0.shape, 23) * o0.free_skeleton_mask()
    x = torch.full((io0.len,), float("nan"), dtype=torch.float64, device=gpu)
    assert g.coarse_solve(io0.to_dev(b), x) == 0
    torch.cuda.synchronize()
    assert rel(io0.to_grid(x), coarse_fd.fd_condensed_solve(o0, b)) <= TOL64
    g.close()


@pytest.mark.parametrize("case", [c for c in CASES if c[1] >= 3], ids=_ids)
def test_vcycle_with_seams(gpu, case):
    g, o = _pair(case)
    io = LevelIO(g, g.num_levels(), o.bc)
    r = synth.random_grid(o.shape, 31) * o.free_skeleton_mask()
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


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_pcg_solve_with_seams(gpu, case):
    """ipCG (Alg. 5), FP64 and mixed: iteration count within one of the
    oracle's, solution to 1e-9, and the oracle's residual of the result."""
    g, o = _pair(case)
    f = synth.random_grid(o.shape, 41)
    ref = solver.solve(o, f, method="kMG", rtol=1e-10, coarse="fd")
    Fh = matfree.condense_rhs(o, o.expand_periodic(f))
    mask = o.free_skeleton_mask()
    for dt in (pmg.F64, pmg.F32):
        u = torch.zeros(o.shape, dtype=torch.float64, device=gpu)
        st = g.pcg_solve(torch.as_tensor(f, device=gpu), u, 1e-10, 100, dt)
        assert st.status == 0 and st.rel_res <= 1e-10
        assert abs(st.iters - ref.iters) <= 1, (dt, st.iters, ref.iters)
        uh = u.cpu().numpy()
        assert rel(uh, ref.u) <= 1e-9
        res = Fh - matfree.condensed_op(o, uh * mask)
        assert np.linalg.norm(res[mask]) <= 2e-10 * np.linalg.norm(Fh[mask])
        assert np.array_equal(uh, o.expand_periodic(uh))
    g.close()


@pytest.mark.parametrize("case", [c for c in CASES if 2 <= c[1] <= 16], ids=_ids)
def test_block_smoother_with_seams(gpu, case):
    """Element-centred blocks (Sec. 3.4) on every level of degree >= 2 with
    Neumann and periodic sides, FP64 and FP32, and a whole solve with them."""
    from oracle import blocks
    g, o = _pair(case)
    g.set_smoother(1)
    for level in range(g.num_levels() + 1):
        io = LevelIO(g, level, o.bc)
        if io.p < 2:
            continue
        ol = o.with_degree(io.p)
        r = synth.random_grid(ol.shape, 71 + level) * ol.free_skeleton_mask()
        ref = blocks.block_smoother(ol, r, 0.8)
        for dt, tdt, tol in ((pmg.F64, torch.float64, TOL64), (pmg.F32, torch.float32, TOL32)):
            z = torch.full((io.len,), float("nan"), dtype=tdt, device=gpu)
            g.schwarz_smooth(level, io.to_dev(r, tdt), z, 0.8, dt)
            torch.cuda.synchronize()
            assert rel(io.to_grid(z), ref) <= tol, (level, dt)
            assert float(z.double().abs().sum()) == pytest.approx(float(np.abs(io.to_grid(z)).sum()), rel=1e-12)
    f = synth.random_grid(o.shape, 75)
    sref = solver.solve(o, f, rtol=1e-10, coarse="fd", smoother="element")
    u = torch.zeros(o.shape, dtype=torch.float64, device=gpu)
    st = g.pcg_solve(torch.as_tensor(f, device=gpu), u, 1e-10, 100, pmg.F64)
    assert st.status == 0 and abs(st.iters - sref.iters) <= 1
    assert rel(u.cpu().numpy(), sref.u) <= 1e-9
    g.close()


@pytest.mark.parametrize("kinds", [(("N", "N"), ("D", "N")), (("N", "D"), "P")])
def test_manufactured_solution(gpu, kinds):
    """sin(x1 + 0.3) periodic on (0, 2 pi) times factors meeting the other
    kinds exactly (cos(pi x): zero slope at both ends; sin(pi x / 2): zero
    at 0, zero slope at 1; cos(pi x / 2): zero slope at 0, zero at 1): the
    solver's nodal error at p = 8 is that of the discretisation."""
    fac = {("N", "N"): (lambda x: np.cos(np.pi * x), np.pi ** 2),
           ("D", "N"): (lambda x: np.sin(np.pi * x / 2), np.pi ** 2 / 4),
           ("N", "D"): (lambda x: np.cos(np.pi * x / 2), np.pi ** 2 / 4),
           "P": (lambda x: np.sin(2 * np.pi * x + 0.5), 4 * np.pi ** 2)}
    (g2, k2), (g3, k3) = fac[kinds[0]], fac[kinds[1]]
    lam = 1.0
    g, o = make_pair((6, 4, 4), 8, lam, 1.0, widths=[np.full(6, 2 * np.pi / 6), np.full(4, 0.25), np.full(4, 0.25)],
                     bc=("P", kinds[0], kinds[1]))
    X3, X2, X1 = o.coords()
    u_ex = np.sin(X1 + 0.3) * g2(X2) * g3(X3)
    f = (1.0 + k2 + k3 + lam) * u_ex
    for dt in (pmg.F64, pmg.F32):
        u = torch.zeros(o.shape, dtype=torch.float64, device=gpu)
        st = g.pcg_solve(torch.as_tensor(f, device=gpu), u, 1e-12, 100, dt)
        assert st.status == 0
        assert np.max(np.abs(u.cpu().numpy() - u_ex)) < 1e-7
    g.close()


def test_unsupported_calls_on_bc_meshes(gpu):
    g, o = make_pair((3, 3, 3), 4, 1.0, bc=("P", "N", "D"))
    for call in (lambda: g.set_coarse_solver(0), lambda: g.set_coarse_mg(1)):
        with pytest.raises(pmg.PmgError) as ei:
            call()
        assert ei.value.code == pmg.EUNSUP
    f = torch.zeros(o.shape, dtype=torch.float64, device=gpu)
    with pytest.raises(pmg.PmgError) as ei:
        g.pcg_solve_dirichlet(f, f.clone(), torch.zeros_like(f))
    assert ei.value.code == pmg.EUNSUP
    # the mesh still solves after the refusals
    st = g.pcg_solve(torch.as_tensor(synth.random_grid(o.shape, 5), device=gpu), f, 1e-10, 50, pmg.F32)
    assert st.status == 0
    g.close()
