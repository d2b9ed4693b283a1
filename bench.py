#!/usr/bin/env python3
"""Benchmark of the condensed p-multigrid Helmholtz solver on one MI355X.

Metric: solved unknowns per second (n_e p^3 / t_solve) to a 1e-10 relative
residual, where one step is one complete solve (condensation, Krylov-
accelerated multigrid iterations of Alg. 5, interior recovery) of the
workload below with its inputs already resident in HBM.  The headline value
is the mixed-precision solver (FP32 V-cycle inside FP64 CG) with the
per-level damping predicted by the trained network (omega = 1 when no
weights are available); the same mixed solver with the paper's omega = 1
and the plain FP64 solver are timed beside it.

Default workload ("c4"): 32 x 32 x 32 elements, p = 8 (16.8M unknowns),
lambda = 0, the anisotropic brick (0, AR) x (0, ceil(AR/2)/2) x (0, 1) with
AR = 1, exact solution a seeded sum of 8 sine modes.  Beside it:
* the whole mixed-precision grid lambda in {0, 1e2, 1e4} x AR in
  {1, 2, 4, 8, 16} at 32^3 elements, p = 8;
* the learned-damping test grid: 24^3 elements, p = 12, held-out
  AR in {3, 6, 12} and lambda h^2 in {0.3, 30, 3e3};
* a p sweep at about 1e7 unknowns (p = 2 .. 48) with the roofline position
  of the star smoother and of the condensed operator at every p;
* a sweep over the unknown count on the paper's runtime test problem.

Roofline: the star smoother (the kernel the method's work count is
dominated by) and the condensed operator, each timed alone with HIP events
on the stream it is launched on; rate / min(peak, HBM bandwidth x
algorithmic intensity).  Parity: every headline solution is checked by the
FP64 oracle at full size (its condensed residual of the returned skeleton
values and its interior recovery from them); the oracle's complete solve of
the same recipe on 16^3 elements gives the relative error of the three GPU
solvers on that sample and the CPU baseline (all host threads, then one
thread, the paper's one-core setting).

  python bench.py [--steps K] [--warmup W] [--workload c4|c2a|c2b|c1|c5|c3p<p>]
  python bench.py --kernel-only     # only the smoother timing loop (profiling)
  python bench.py --op-only         # only the condensed-operator timing loop
  python bench.py --sweep-kernels   # smoother and operator timing at every sweep p
  python bench.py --copy-only       # one device copy of 512 MiB (counter scale)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3}   # TFLOP/s, MI355X dense vector / matrix
HBM_PEAK = 8000.0                     # GB/s
ROOFLINE_KERNEL = "k_smoother_mfma<float, 1>"

# HBM bytes per launch of the roofline kernel at the default workload, from
# two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of
# "python bench.py --kernel-only", each scaled by the same counter's reading
# for a plain 512 MiB device copy; valid only for the kernel source whose
# hash (kernels_sha1 below) is recorded with it and for the workload named.
TRAFFIC = {"kernels_sha1": "f9b1519be075504aabd094088980a800f74ac8db", "workload": "c4",
           "bytes_per_launch": 145595001}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernels_sha1():
    """Hash of the source the roofline kernel is built from: the shared
    helpers at the top of the kernel file, the matrix-core smoother itself,
    its argument types (Layout, LevelTabs) and the compiler flags (edits
    elsewhere leave its traffic record valid)."""
    csrc = os.path.join(ROOT, "paper_1808_03595_amd", "csrc")
    with open(os.path.join(csrc, "pmg_kernels.hip")) as fh:
        src = fh.read()
    head = src[:src.index("template <typename T>\n__device__ inline void add_out")]
    body = src[src.index("// Matrix-core star smoother for n_S"):src.index("// Star smoother for small stars")]
    with open(os.path.join(csrc, "pmg_internal.h")) as fh:
        hdr = fh.read()
    hdr = hdr[hdr.index("struct Layout {"):hdr.index("// Working-set sizes")]  # the kernel's argument types
    from paper_1808_03595_amd import build as pbuild
    h = hashlib.sha1()
    for part in (head, body, hdr, " ".join(pbuild.FLAGS)):
        h.update(part.encode())
    return h.hexdigest()


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def brick(n, p, lam, ar, seed=0):
    """Anisotropic brick recipe (Sec. 5.3 scaled to unit height), n^3 uniform elements."""
    import synth
    (hx, hy, hz), lengths = synth.anisotropic_widths(n, ar)
    return dict(n=(n, n, n), p=p, lam=lam, widths=(hx, hy, hz), lengths=lengths, seed=seed, modes="sine8",
                desc=(f"{n}x{n}x{n} elements, p={p}, lambda={lam:g}, brick (0,{lengths[0]:g})x(0,{lengths[1]:g})"
                      f"x(0,1) (AR {ar:g}), 8 sine modes seed {seed}"))


def stretched(n, p, lam, alpha, seed=0):
    """Unit cube, widths h_k ~ alpha^k in every direction (Sec. 5.4)."""
    import synth
    h = synth.stretched_widths(n, alpha)
    return dict(n=(n, n, n), p=p, lam=lam, widths=(h, h, h), lengths=(1.0, 1.0, 1.0), seed=seed, modes="sine8",
                alpha=alpha, desc=(f"{n}x{n}x{n} elements, p={p}, lambda={lam:g}, unit cube stretched alpha={alpha:.4f} "
                      f"(AR {alpha ** (n - 1):.1f}), 8 sine modes seed {seed}"))


def workload(name):
    import numpy as np
    if name == "c4":
        return brick(32, 8, 0.0, 1)
    if name == "c5":
        # one held-out point of the learned-damping test: AR 6, lambda h^2 = 30
        w = brick(24, 12, 0.0, 6)
        hmin = min(float(np.min(h)) for h in w["widths"])
        return brick(24, 12, 30.0 / hmin ** 2, 6)
    if name == "c2a":
        return stretched(16, 8, 1.0, 8.0 ** (1.0 / 15.0))
    if name == "c2b":
        return stretched(8, 16, 1.0, 8.0 ** (1.0 / 7.0))
    if name == "c1":
        w = stretched(4, 4, 1.0, 1.0)
        w["modes"] = "product"
        w["desc"] = "4x4x4 elements, p=4, lambda=1, unit cube, u = sin(pi x) sin(pi y) sin(pi z)"
        return w
    if name.startswith("c3p") and name[3:].isdigit():  # one point of the p sweep
        p = int(name[3:])
        return stretched(int(round(215.44 / p)), p, 1.0, 1.0)
    raise SystemExit(f"unknown workload {name}")


def is_uniform(wl):
    import numpy as np
    return all(float(np.ptp(h)) <= 1e-12 * float(np.max(h)) for h in wl["widths"])


def create(pmg, wl):
    hx, hy, hz = wl["widths"]
    return pmg.create_mesh_widths(hx, hy, hz, wl["p"], wl["lam"])


def make_rhs(g, wl, torch, synth, dev):
    x1, x2, x3 = (torch.tensor(c, dtype=torch.float64, device=dev) for c in g.grid_coords())
    k, a = synth.product_mode() if wl["modes"] == "product" else synth.sine_modes(wl["seed"])
    u, f = synth.sine_solution(k, a, wl["lengths"], x1[None, None, :], x2[None, :, None],
                               x3[:, None, None], wl["lam"], xp=torch)
    shape = g.grid_shape()
    return u.expand(shape).contiguous(), f.expand(shape).contiguous()


def coarse_levels(p, uniform, ne):
    """Degree-1 levels below p_0 = 2 (Sec. 4.2's low-order coarse grid) for
    degree p on a mesh of ne elements (uniform: equal widths per direction).

    Measured on one MI355X (whole solves to 1e-10): at p <= 4 the coarse
    problem is most of the mesh and six levels win.  At p = 8 one level wins
    on uniform meshes of 16^3 elements or more (the paper's test problem at
    16^3..40^3 elements: 1.2-2.1x; the p = 8 sweep point: 1.28x; the 32^3
    bricks of AR 1..16 at every lambda) and loses on 8^3 elements and on
    stretched meshes (aspect ratio 8: 7 -> 10 outer iterations).  At p >= 12
    (meshes of 18^3 elements or fewer in the sweep, deeper p-hierarchies) it
    loses 0-25 %.
    """
    if p <= 4:
        return 6
    return 1 if (p <= 8 and uniform and ne >= 16 ** 3) else 0


# coarse solver of every solve: "fd" (exact solve by fast diagonalization of
# the whole coarse mesh) or "cg" (the paper's Jacobi CG on p_0 = 2, with the
# degree-1 levels of coarse_levels below it)
COARSE = {"kind": "fd", "level": "auto"}


def configure_coarse(g, wl, coarse_rtol):
    """Set up the coarse solver of mesh g for workload wl; returns its
    description and the oracle's matching keyword arguments."""
    g.set_cycle(0, coarse_rtol, 5000)
    if COARSE["kind"] == "fd":
        g.set_coarse_mg(0, 0.8, 2)
        g.set_coarse_solver(1)
        return "exact (fast diagonalization)", {"coarse": "fd"}
    g.set_coarse_solver(0)
    n = wl["n"]
    hmg = coarse_levels(wl["p"], is_uniform(wl), n[0] * n[1] * n[2])
    g.set_coarse_mg(hmg, 0.8, 2)
    desc = (f"{hmg} degree-1 level(s) + " if hmg else "") + f"Jacobi CG to rel. {coarse_rtol:g}"
    kw = {"coarse_rtol": coarse_rtol, "coarse_maxit": 5000}
    if hmg:
        kw.update(hmg_levels=hmg, hmg_omega=0.8, hmg_nu=2)
    return desc, kw


FD_MAX = 200   # largest fast-diagonalization size n_d p_k per direction a coarse level may have


def coarse_candidates(g):
    """p-levels k whose condensed system the exact coarse solve may invert:
    0 <= k < L (at least one smoothed level stays) with n_d p_k <= FD_MAX."""
    L = g.num_levels()
    return [k for k in range(max(L, 1)) if max(g.n) * g.level_degree(k) <= FD_MAX] or [0]


def tune_coarse_level(g, solve, torch, reps=2):
    """The exact coarse level whose whole solve measures fastest (one warm-up
    and `reps` timed solves per candidate, outside every timed region);
    returns (level, {level: ms})."""
    if COARSE["kind"] != "fd" or g.num_levels() == 0:
        return 0, {}
    if COARSE["level"] != "auto":
        return int(COARSE["level"]), {}
    ms = {}
    for k in coarse_candidates(g):
        g.set_coarse_level(k)
        solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            solve()
        torch.cuda.synchronize()
        ms[k] = (time.perf_counter() - t0) / reps * 1e3
    best = min(ms, key=ms.get)
    g.set_coarse_level(best)
    return best, ms


def learned_damping(wl, L):
    """omega predicted by the trained network for this mesh, or None."""
    from paper_1808_03595_amd.learn import DampingMLP, predict_damping
    model = DampingMLP.load()
    if model is None or L == 0:
        return None
    hx, hy, hz = wl["widths"]
    return predict_damping(model, wl["p"], wl["lam"], hx, hy, hz, L)


# ---------------------------------------------------------------------------
# algorithmic work (Sec. 3.2 and Sec. 4.2 counts)
# ---------------------------------------------------------------------------

def n_stars(n):
    """All mesh vertices except the 8 domain corners (three Dirichlet planes)."""
    return (n[0] + 1) * (n[1] + 1) * (n[2] + 1) - 8


def smoother_flops(n, p):
    """One smoother application: 37 n_S^3 per star, n_S = 2p - 1 (Sec. 3.2)."""
    return 37.0 * (2 * p - 1) ** 3 * n_stars(n)


def op_flops(n, p):
    """One condensed-operator application: 73 (p-1)^3 + 24 p^3 per element."""
    return (73.0 * (p - 1) ** 3 + 24.0 * p ** 3) * n[0] * n[1] * n[2]


def n_hat(n, p):
    """Unique condensed unknowns (homogeneous Dirichlet)."""
    return (n[0] * p - 1) * (n[1] * p - 1) * (n[2] * p - 1) - n[0] * n[1] * n[2] * (p - 1) ** 3


def vec_bytes(n, p, tsize):
    """Algorithmic HBM bytes of K1 or K2: read the input and write the output once."""
    return 2.0 * n_hat(n, p) * tsize


def roofline(flops, nbytes, t, prec):
    """Position of a kernel against min(peak, HBM bandwidth x intensity)."""
    peak = PEAK[prec]
    bw_bound = HBM_PEAK * 1e9 * flops / nbytes / 1e12   # TFLOP/s the HBM roof allows
    if bw_bound < peak:
        ach = nbytes / t / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK, "unit": "GB/s", "frac": ach / HBM_PEAK,
                "us_per_launch": t * 1e6}
    ach = flops / t / 1e12
    return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
            "us_per_launch": t * 1e6}


def smoother_kernel(p, t):
    """The smoother kernel that degree p runs (t: "float" or "double")."""
    nS = 2 * p - 1
    if nS <= 3:
        return f"k_smoother_small<{t}, 3>"
    if nS <= 7:
        return f"k_smoother_small<{t}, 8>"
    if nS <= 16:
        return f"k_smoother_mfma<{t}, 1>"
    return f"k_star_gemm<{t}, ...> + k_star_eigen<{t}> (batched)"


def op_kernel(p, t):
    """The condensed-operator kernels that degree p runs."""
    if p == 2:
        return f"k_centre_t<{t}> + k_condensed_op_box2<{t}>"
    if p <= 8 or p in (12, 16):
        return f"k_condensed_op_w<{t}, {p}> + k_gather_elem<{t}, {p}>"
    if p <= 16:
        return f"k_condensed_op<{t}> + k_gather_elem"
    return f"k_op_big_fwd/contract/bwd<{t}> + k_gather_elem"


def _timed(torch, fn, reps):
    s = torch.cuda.current_stream()
    for _ in range(3):
        fn(s)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn(s)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def _level_vector(g, torch, dev, dtype, level):
    import paper_1808_03595_amd as pmg
    n = g.skeleton_len(level)
    tdt = torch.float64 if dtype == pmg.F64 else torch.float32
    r = torch.randn(n, dtype=tdt, device=dev)
    if level == g.num_levels():          # zero the unused slots of r
        tmp = torch.empty(g.grid_shape(), dtype=torch.float64, device=dev)
        g.skeleton_to_grid(r, tmp, dtype)
        g.grid_to_skeleton(tmp, r, dtype)
    return r


def time_smoother(g, torch, dev, dtype, reps=50):
    """Average duration of one smoothing update u += S(r) on the finest
    level, HIP events recorded on the stream the kernel is launched on."""
    L = g.num_levels()
    r = _level_vector(g, torch, dev, dtype, L)
    u = torch.zeros_like(r)
    return _timed(torch, lambda s: g.schwarz_smooth_add(L, r, u, 1.0, dtype, stream=s), reps)


def time_operator(g, torch, dev, dtype, reps=50):
    """Average duration of one condensed-operator application y = H u on the
    finest level (element kernels and the gather), HIP events on its stream."""
    L = g.num_levels()
    u = _level_vector(g, torch, dev, dtype, L)
    y = torch.empty_like(u)
    return _timed(torch, lambda s: g.apply_condensed_op(L, u, y, dtype, stream=s), reps)


def kernel_rooflines(g, torch, dev, n, p, reps=50):
    """Smoother and operator at the finest level, FP32 and FP64."""
    import paper_1808_03595_amd as pmg
    out = {}
    for prec, dtype, ts in (("f32", pmg.F32, 4), ("f64", pmg.F64, 8)):
        t_s = time_smoother(g, torch, dev, dtype, reps)
        t_o = time_operator(g, torch, dev, dtype, reps)
        tname = "float" if prec == "f32" else "double"
        rs = roofline(smoother_flops(n, p), vec_bytes(n, p, ts), t_s, prec)
        rs["kernel"] = smoother_kernel(p, tname)
        ro = roofline(op_flops(n, p), vec_bytes(n, p, ts), t_o, prec)
        ro["kernel"] = op_kernel(p, tname)
        out[prec] = {"smoother": rs, "operator": ro}
    return out


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

def timed_solves(g, f, u, dtype, omega, steps, warm, torch, maxit=300):
    g.set_damping(omega)
    for _ in range(warm):
        g.pcg_solve(f, u, 1e-10, maxit, dtype)
    torch.cuda.synchronize()
    ts = []
    st = None
    for _ in range(steps):
        t0 = time.perf_counter()
        st = g.pcg_solve(f, u, 1e-10, maxit, dtype)   # synchronises before it returns
        ts.append(time.perf_counter() - t0)
    return sum(ts) / len(ts), min(ts), st


def solver_row(g, wl, torch, synth, dev, steps, warm, with_omega1=False, keep=False):
    """FP64, mixed + learned (and mixed with omega = 1) on one workload."""
    import paper_1808_03595_amd as pmg
    n, p = wl["n"], wl["p"]
    L = g.num_levels()
    u_ex, f = make_rhs(g, wl, torch, synth, dev)
    u = torch.zeros_like(f)
    ndof = n[0] * n[1] * n[2] * p ** 3
    omega = learned_damping(wl, L)
    runs = [("fp64", pmg.F64, None), ("mixed_learned", pmg.F32, omega)]
    if with_omega1:
        runs.insert(1, ("mixed_omega1", pmg.F32, None))
    row, sols = {}, {}
    for name, dtype, om in runs:
        g.set_damping(om)
        cl, cand = tune_coarse_level(g, lambda: g.pcg_solve(f, u, 1e-10, 300, dtype), torch)
        mean, best, st = timed_solves(g, f, u, dtype, om, steps, warm, torch)
        err = (torch.linalg.vector_norm(u - u_ex) / torch.linalg.vector_norm(u_ex)).item()
        row[name] = {"unknowns_per_s": ndof / mean, "ms": mean * 1e3, "ms_min": best * 1e3,
                     "iters": st.iters, "coarse_iters": st.coarse_iters, "rel_res": st.rel_res,
                     "status": st.status, "rel_err_vs_exact": err,
                     "coarse_level": cl, "coarse_degree": g.level_degree(cl),
                     "coarse_level_ms": {str(k): v for k, v in cand.items()}}
        if keep:
            sols[name] = u.cpu().numpy()
    g.set_damping(None)
    if COARSE["kind"] == "fd":
        g.set_coarse_level(0)
    row["omega"] = omega
    return row, ndof, (f.cpu().numpy() if keep else None), sols


def c4_grid(torch, pmg, synth, dev, coarse_rtol, steps, warm):
    """Mixed precision + learned damping against FP64 at 32^3 elements, p = 8,
    lambda in {0, 1e2, 1e4} x AR in {1, 2, 4, 8, 16} (anisotropic bricks)."""
    out = []
    for lam in (0.0, 1e2, 1e4):
        for ar in (1, 2, 4, 8, 16):
            wl = brick(32, 8, lam, ar)
            g = create(pmg, wl)
            cdesc, _ = configure_coarse(g, wl, coarse_rtol)
            row, ndof, _, _ = solver_row(g, wl, torch, synth, dev, steps, warm)
            row.update({"lambda": lam, "ar": ar, "ndof": ndof, "coarse": cdesc,
                        "parity": "rel_res recomputed by the solver; oracle check at the headline only"})
            log(f"[bench] c4 grid lambda={lam:g} AR={ar}: fp64 {row['fp64']['ms']:.2f} ms "
                f"({row['fp64']['iters']} it), mixed+learned {row['mixed_learned']['ms']:.2f} ms "
                f"({row['mixed_learned']['iters']} it)")
            out.append(row)
            g.close()
            torch.cuda.empty_cache()
    return out


def c5_grid(torch, pmg, synth, dev, coarse_rtol, steps, warm):
    """Learned damping on the held-out test meshes: 24^3 elements, p = 12,
    AR in {3, 6, 12}, lambda h_min^2 in {0.3, 30, 3e3}; mixed + learned
    against mixed with omega = 1 and FP64."""
    import numpy as np
    out = []
    for ar in (3, 6, 12):
        for lh2 in (0.3, 30.0, 3e3):
            w0 = brick(24, 12, 0.0, ar)
            hmin = min(float(np.min(h)) for h in w0["widths"])
            wl = brick(24, 12, lh2 / hmin ** 2, ar)
            g = create(pmg, wl)
            cdesc, _ = configure_coarse(g, wl, coarse_rtol)
            row, ndof, _, _ = solver_row(g, wl, torch, synth, dev, steps, warm, with_omega1=True)
            row.update({"ar": ar, "lambda_h2": lh2, "lambda": wl["lam"], "ndof": ndof, "coarse": cdesc})
            log(f"[bench] c5 AR={ar} lambda h^2={lh2:g}: mixed omega=1 {row['mixed_omega1']['ms']:.2f} ms "
                f"({row['mixed_omega1']['iters']} it), learned {row['mixed_learned']['ms']:.2f} ms "
                f"({row['mixed_learned']['iters']} it)")
            out.append(row)
            g.close()
            torch.cuda.empty_cache()
    tot = {k: sum(r[k]["iters"] for r in out) for k in ("fp64", "mixed_omega1", "mixed_learned")}
    ms = {k: sum(r[k]["ms"] for r in out) for k in ("fp64", "mixed_omega1", "mixed_learned")}
    return {"rows": out, "total_iters": tot, "total_ms": ms}


SWEEP = (2, 4, 8, 12, 16, 24, 32, 48)


def p_sweep(torch, pmg, synth, dev, coarse_rtol, steps, warm):
    """Unknowns/s versus p at about 1e7 unknowns (n = round(215.44 / p)
    elements per direction, uniform, lambda = 1, 8 sine modes), plain FP64
    and mixed precision with the learned damping, with the smoother's and
    the operator's roofline position at every p."""
    out = []
    for p in SWEEP:
        wl = workload(f"c3p{p}")
        nn = wl["n"][0]
        g = create(pmg, wl)
        cdesc, _ = configure_coarse(g, wl, coarse_rtol)
        L = g.num_levels()
        row, ndof, _, _ = solver_row(g, wl, torch, synth, dev, steps, warm)
        row.update({"p": p, "n": nn, "ndof": ndof, "levels": L + 1, "coarse": cdesc,
                    "parity": "parity unpinned at this size (no oracle solve); rel_res from the solver"})
        if L > 0:
            row["kernels"] = kernel_rooflines(g, torch, dev, wl["n"], p)
        log(f"[bench] sweep p={p} n={nn}: fp64 {row['fp64']['ms']:.1f} ms ({row['fp64']['iters']} it), "
            f"mixed+learned {row['mixed_learned']['ms']:.1f} ms ({row['mixed_learned']['iters']} it)")
        out.append(row)
        g.close()
        torch.cuda.empty_cache()
    return out


NSWEEP = (8, 16, 24, 32, 40)


def n_sweep(torch, pmg, synth, dev, coarse_rtol, steps, warm):
    """Runtime versus the number of unknowns (the linear-scaling claim,
    Sec. 5.2): the paper's runtime test problem on (0, 2 pi)^3 (manufactured
    solution with k = 5, lambda = 0, its values as inhomogeneous Dirichlet
    data on the whole boundary), p = 8 on n^3 uniform elements, plain FP64
    and mixed precision with the learned damping."""
    out = []
    p = 8
    for nn in NSWEEP:
        h = [2.0 * math.pi / nn] * nn
        g = pmg.create_mesh_widths(h, h, h, p, 0.0)
        wln = dict(n=(nn, nn, nn), p=p, lam=0.0, widths=(h, h, h))
        cdesc, _ = configure_coarse(g, wln, coarse_rtol)
        L = g.num_levels()
        x1, x2, x3 = (torch.tensor(c, dtype=torch.float64, device=dev) for c in g.grid_coords())
        u_ex, f = synth.paper_test_solution(5.0, 0.0, x1[None, None, :], x2[None, :, None],
                                            x3[:, None, None], xp=torch)
        u_ex, f = u_ex.contiguous(), f.contiguous()
        u = torch.zeros_like(f)
        ndof = nn ** 3 * p ** 3
        row = {"n": nn, "p": p, "ndof": ndof, "coarse": cdesc,
               "parity": "parity unpinned at this size (no oracle solve); rel_res from the solver"}
        omega = learned_damping(wln, L)
        for name, dtype, om in (("fp64", pmg.F64, None), ("mixed_learned", pmg.F32, omega)):
            g.set_damping(om)
            cl, _ = tune_coarse_level(g, lambda: g.pcg_solve_dirichlet(f, u_ex, u, 1e-10, 300, dtype), torch)
            for _ in range(warm):
                g.pcg_solve_dirichlet(f, u_ex, u, 1e-10, 300, dtype)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                st = g.pcg_solve_dirichlet(f, u_ex, u, 1e-10, 300, dtype)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            err = (u - u_ex).abs().max().item()
            row[name] = {"ms": dt * 1e3, "iters": st.iters, "ns_per_unknown": dt * 1e9 / ndof,
                         "coarse_level": cl, "coarse_degree": g.level_degree(cl),
                         "ns_per_unknown_iter": dt * 1e9 / ndof / max(st.iters, 1),
                         "coarse_iters": st.coarse_iters, "rel_res": st.rel_res,
                         "max_err_vs_exact": err, "status": st.status}
        log(f"[bench] n sweep n={nn} ({ndof / 1e6:.1f}M unknowns): fp64 {row['fp64']['ms']:.1f} ms "
            f"({row['fp64']['iters']} it), mixed+learned {row['mixed_learned']['ms']:.1f} ms "
            f"({row['mixed_learned']['iters']} it)")
        out.append(row)
        g.close()
        del u, f, u_ex
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# oracle: parity of the headline solutions and the CPU baseline
# ---------------------------------------------------------------------------

def oracle_mesh(wl):
    from oracle import mesh as omesh
    hx, hy, hz = wl["widths"]
    return omesh.Mesh(hx, hy, hz, wl["p"], wl["lam"])


def oracle_check(wl, f, sols):
    """Full-size parity of GPU solutions: the oracle's condensed residual of
    the returned skeleton values (relative to its condensed right-hand side)
    and the relative difference between the returned grid and the oracle's
    interior recovery from those skeleton values."""
    import numpy as np
    from oracle import matfree
    o = oracle_mesh(wl)
    t0 = time.perf_counter()
    Fh = matfree.condense_rhs(o, f)
    mask = o.free_skeleton_mask()
    nF = float(np.linalg.norm(Fh[mask]))
    out = {}
    for name, u in sols.items():
        uh = u * mask
        res = float(np.linalg.norm((Fh - matfree.condensed_op(o, uh))[mask])) / nF
        rec = matfree.recover_interior(o, f, uh)
        out[name] = {"oracle_rel_res": res,
                     "rel_diff_vs_oracle_recovery": float(np.linalg.norm(u - rec) / np.linalg.norm(rec))}
        log(f"[bench] oracle check {name}: residual {res:.2e}, recovery {out[name]['rel_diff_vs_oracle_recovery']:.2e}")
    out["seconds"] = time.perf_counter() - t0
    return out


def oracle_solve(wl, f, ckw):
    """The FP64 oracle's complete solve (condensation, ipCG to 1e-10 with the
    same coarse solver, recovery); returns (u, iters, s)."""
    from oracle import solver
    o = oracle_mesh(wl)
    t0 = time.perf_counter()
    res = solver.solve(o, f, method="kMG", rtol=1e-10, **ckw)
    return res.u, res.iters, time.perf_counter() - t0


def cpu_parity_and_baseline(wl_sample, wl_small, torch, pmg, synth, dev, coarse_rtol, steps, warm):
    """Oracle solve of the sample (all host threads) -> CPU baseline and the
    GPU solvers' relative error against it; 1-thread oracle solve of
    wl_small (the paper quotes one-core runtimes)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    threads = len(os.sched_getaffinity(0))
    g = create(pmg, wl_sample)
    _, ckw = configure_coarse(g, wl_sample, coarse_rtol)
    row, ndof, f, sols = solver_row(g, wl_sample, torch, synth, dev, steps, warm, with_omega1=True, keep=True)
    g.close()
    u_or, it_or, t_or = oracle_solve(wl_sample, f, ckw)
    nr = float(np.linalg.norm(u_or))
    errs = {k: float(np.linalg.norm(v - u_or)) / nr for k, v in sols.items()}
    log(f"[bench] oracle sample solve: {t_or:.1f} s on {threads} threads, {it_or} iterations; "
        f"GPU rel. errors {errs}")
    g = create(pmg, wl_small)
    _, fs = make_rhs(g, wl_small, torch, synth, dev)
    fs = fs.cpu().numpy()
    _, ckw_s = configure_coarse(g, wl_small, coarse_rtol)
    g.close()
    ne_s = wl_small["n"][0] * wl_small["n"][1] * wl_small["n"][2]
    with threadpool_limits(limits=1):
        _, it1, t1 = oracle_solve(wl_small, fs, ckw_s)
    ndof_s = ne_s * wl_small["p"] ** 3
    log(f"[bench] oracle 1-thread solve of {wl_small['desc']}: {t1:.1f} s, {it1} iterations")
    return {
        "sample": wl_sample["desc"], "ndof": ndof, "oracle_iters": it_or, "oracle_s": t_or,
        "threads": threads, "gpu": row, "rel_err_vs_oracle": errs,
        "one_thread": {"sample": wl_small["desc"], "ndof": ndof_s, "s": t1, "iters": it1,
                       "unknowns_per_s": ndof_s / t1},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle parity checks and CPU baseline")
    ap.add_argument("--coarse-rtol", type=float, default=3e-2,
                    help="relative tolerance of the coarse CG (the paper leaves it open)")
    ap.add_argument("--coarse", choices=["fd", "cg"], default="fd",
                    help="coarse solver: exact fast-diagonalization solve (default) or the paper's Jacobi CG "
                         "(with degree-1 levels below p_0 = 2: 6 at p <= 4; 1 at p <= 8 on uniform meshes of "
                         ">= 16^3 elements; else none)")
    ap.add_argument("--coarse-level", default="auto",
                    help="p-level of the exact coarse solve: 'auto' (the fastest of the levels below the finest "
                         "whose fast-diagonalization size is at most 200 per direction, measured per solver "
                         "before its timed solves) or a level index")
    ap.add_argument("--kernel-only", action="store_true",
                    help="run only the smoother timing loop (for counter profiles)")
    ap.add_argument("--op-only", action="store_true",
                    help="run only the condensed-operator timing loop (for counter profiles)")
    ap.add_argument("--sweep-kernels", action="store_true",
                    help="time only the smoother and the operator at every p of the sweep")
    ap.add_argument("--sweep-p", type=int, default=None,
                    help="with --sweep-kernels: only this degree of the sweep")
    ap.add_argument("--copy-only", action="store_true",
                    help="run one 512 MiB device copy (scale of the byte counters)")
    ap.add_argument("--profile-solve", action="store_true",
                    help="run only the headline solver (mixed precision, learned damping): warm-up and timed "
                         "solves, for kernel-share profiles")
    ap.add_argument("--no-sweep", action="store_true", help="skip the p and n sweeps")
    ap.add_argument("--no-grids", action="store_true", help="skip the 32^3 and the learned-damping grids")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the solver is a single-GPU build; see the sharding notes in the design document)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1808_03595_amd as pmg
    import synth

    dev = torch.device("cuda:0")
    if args.copy_only:
        a = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copied 512 MiB")
        return
    if args.sweep_kernels:
        for p in (SWEEP if args.sweep_p is None else (args.sweep_p,)):
            wl = workload(f"c3p{p}")
            g = create(pmg, wl)
            if g.num_levels() > 0:
                r = kernel_rooflines(g, torch, dev, wl["n"], p, reps=100)
                log(f"[bench] p={p}: " + json.dumps(r))
            g.close()
        return
    wl = workload(args.workload)
    n, p = wl["n"], wl["p"]
    ne = n[0] * n[1] * n[2]
    g = create(pmg, wl)
    L = g.num_levels()
    if args.kernel_only or args.op_only:
        fn = time_smoother if args.kernel_only else time_operator
        t = fn(g, torch, dev, pmg.F32, reps=100)
        log(f"[bench] {'smoother' if args.kernel_only else 'operator'} f32: {t * 1e6:.2f} us per launch")
        return
    COARSE["kind"] = args.coarse
    COARSE["level"] = args.coarse_level
    cdesc, _ = configure_coarse(g, wl, args.coarse_rtol)
    log(f"[bench] workload {args.workload}: {wl['desc']}; coarse solver: {cdesc}")
    if args.profile_solve:
        u_ex, f = make_rhs(g, wl, torch, synth, dev)
        u = torch.zeros_like(f)
        om = learned_damping(wl, L)
        g.set_damping(om)
        cl, _ = tune_coarse_level(g, lambda: g.pcg_solve(f, u, 1e-10, 300, pmg.F32), torch)
        mean, best, st = timed_solves(g, f, u, pmg.F32, om, args.steps, args.warmup, torch)
        log(f"[bench] mixed learned: {mean * 1e3:.2f} ms/solve iters={st.iters} rel_res={st.rel_res:.2e} "
            f"coarse level {cl} (p = {g.level_degree(cl)})")
        return
    head, ndof, f_head, sols = solver_row(g, wl, torch, synth, dev, args.steps, args.warmup,
                                          with_omega1=True, keep=not args.no_cpu)
    for k in ("fp64", "mixed_omega1", "mixed_learned"):
        r = head[k]
        log(f"[bench] {k}: {r['ms']:.2f} ms/solve (min {r['ms_min']:.2f}) iters={r['iters']} "
            f"rel_res={r['rel_res']:.2e} coarse_iters={r['coarse_iters']} err_vs_exact={r['rel_err_vs_exact']:.2e} "
            f"coarse level {r['coarse_level']} (p = {r['coarse_degree']}) {r['coarse_level_ms']}")
    mixed = head["mixed_learned"]

    roof, kern = None, None
    if L > 0:   # p_0 = 2 alone has no smoothed level
        kern = kernel_rooflines(g, torch, dev, n, p, reps=100)
        rs = kern["f32"]["smoother"]
        traffic = None
        if TRAFFIC["kernels_sha1"] == kernels_sha1() and args.workload == TRAFFIC["workload"]:
            traffic = TRAFFIC["bytes_per_launch"]
        roof = {"bound": rs["bound"], "kernel": rs["kernel"], "achieved": rs["achieved"], "peak": rs["peak"],
                "unit": rs["unit"], "frac": rs["frac"], "traffic": traffic,
                "algorithmic_bytes": vec_bytes(n, p, 4), "flops_per_launch": smoother_flops(n, p),
                "us_per_launch": rs["us_per_launch"], "distance_to_50pct_target": 0.5 - rs["frac"]}
        log(f"[bench] kernels: " + json.dumps(kern))
    g.close()
    torch.cuda.empty_cache()

    grid4 = grid5 = None
    if not args.no_grids:
        grid4 = c4_grid(torch, pmg, synth, dev, args.coarse_rtol, args.steps, args.warmup)
        grid5 = c5_grid(torch, pmg, synth, dev, args.coarse_rtol, args.steps, args.warmup)
    sweep = nsweep = None
    if not args.no_sweep:
        sweep = p_sweep(torch, pmg, synth, dev, args.coarse_rtol, args.steps, args.warmup)
        nsweep = n_sweep(torch, pmg, synth, dev, args.coarse_rtol, args.steps, args.warmup)

    cpu = parity = None
    if not args.no_cpu:
        parity = {"full_size": oracle_check(wl, f_head, sols)}
        # the oracle's complete solve of the same recipe on a smaller mesh
        sample = _resize(wl, tuple(max(2, k // 2) for k in n) if ne > 16 ** 3 else n)
        cb = cpu_parity_and_baseline(sample, sample, torch, pmg, synth, dev, args.coarse_rtol, args.steps,
                                     args.warmup)
        parity["sample"] = {"workload": cb["sample"], "rel_err_vs_oracle": cb["rel_err_vs_oracle"],
                            "oracle_iters": cb["oracle_iters"], "gpu": cb["gpu"]}
        cpu = {"value": cb["ndof"] / cb["oracle_s"], "unit": "unknowns/s", "cores": cb["threads"],
               "kind": "oracle",
               "sample": (f"the FP64 oracle's complete solve of the same recipe on a smaller mesh: {cb['sample']} "
                          f"({cb['oracle_iters']} ipCG iterations to 1e-10), timed once: {cb['oracle_s']:.1f} s"),
               "one_thread": cb["one_thread"]}

    # what the learned damping gains over the paper's omega = 1 on this workload
    lo, ll = head["mixed_omega1"], head["mixed_learned"]
    gain = lo["iters"] - ll["iters"]
    learned_vs = {"iters_learned": ll["iters"], "iters_omega1": lo["iters"], "ms_learned": ll["ms"],
                  "ms_omega1": lo["ms"],
                  "summary": ("the learned damping gains no iteration over omega = 1 on this workload"
                              if gain <= 0 else
                              f"the learned damping saves {gain} iteration(s) over omega = 1 on this workload")}
    log(f"[bench] learned damping vs omega = 1: {learned_vs['summary']} "
        f"({ll['iters']} / {lo['iters']} iterations, {ll['ms']:.2f} / {lo['ms']:.2f} ms)")
    line = {
        "metric": "solved unknowns/s to 1e-10 residual vs p; FP32-MG+learned vs plain FP64",
        "value": mixed["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-vcycle/f64-cg",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "ndof": ndof, "iters": mixed["iters"], "rel_res": mixed["rel_res"],
                   "damping": "learned" if head["omega"] is not None else "omega=1 (paper)",
                   "omega": head["omega"],
                   "coarse": cdesc,
                   "coarse_level": mixed["coarse_level"], "coarse_degree": mixed["coarse_degree"],
                   "coarse_iters_per_solve": mixed["coarse_iters"],
                   "solvers": {k: head[k] for k in ("fp64", "mixed_omega1", "mixed_learned")},
                   "learned_vs_omega1": learned_vs},
        "roofline": roof,
        "kernels": kern,
        "cpu_baseline": cpu,
        "parity": parity,
        "c4_grid": grid4,
        "c5_learned": grid5,
        "p_sweep": sweep,
        "n_sweep": nsweep,
    }
    print(json.dumps(line), flush=True)


def _resize(wl, n):
    """The same recipe on n elements per direction."""
    nn = n[0]
    if wl["modes"] == "product":
        w = stretched(nn, wl["p"], wl["lam"], 1.0)
        w.update(modes="product", desc=wl["desc"].replace(f"{wl['n'][0]}x{wl['n'][1]}x{wl['n'][2]}",
                                                          f"{nn}x{nn}x{nn}"))
        return w
    lx = wl["lengths"]
    if lx == (1.0, 1.0, 1.0):
        h = wl["widths"][0]
        alpha = float(h[1] / h[0]) if len(h) > 1 else 1.0
        return stretched(nn, wl["p"], wl["lam"], alpha ** ((len(h) - 1) / max(nn - 1, 1)), wl["seed"])
    ar = lx[0]
    return brick(nn, wl["p"], wl["lam"], ar, wl["seed"])


if __name__ == "__main__":
    main()
