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

Default workload: 16 x 16 x 16 elements, p = 8 (levels 2, 4, 8), lambda = 1,
geometric stretching up to aspect ratio 8 (alpha = 8^(1/15)), exact solution
a seeded sum of 8 sine modes.

Also reported: the roofline position of the star smoother (the kernel the
method's work count is dominated by), timed alone with HIP events on its
stream, with the HBM traffic measured by rocprofv3 counters; and the CPU
oracle timed on a bounded sample of the same workload on the host cores.

  python bench.py [--steps K] [--warmup W] [--workload c2a|c2b|c1]
  python bench.py --kernel-only     # only the smoother timing loop (profiling)
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
# hash (kernels_sha1 below) is recorded with it.
TRAFFIC = {"kernels_sha1": "34fdb85e3c6873bd7bb089d230a1439904f3ca61", "bytes_per_launch": 19049538}


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


def workload(name):
    if name == "c2a":
        return dict(n=(16, 16, 16), p=8, lam=1.0, alpha=8.0 ** (1.0 / 15.0), seed=0)
    if name == "c2b":
        return dict(n=(8, 8, 8), p=16, lam=1.0, alpha=8.0 ** (1.0 / 7.0), seed=0)
    if name == "c1":
        return dict(n=(4, 4, 4), p=4, lam=1.0, alpha=1.0, seed=0)
    if name.startswith("c3p") and name[3:].isdigit():  # one point of the p sweep
        p = int(name[3:])
        nn = int(round(215.44 / p))
        return dict(n=(nn, nn, nn), p=p, lam=1.0, alpha=1.0, seed=0)
    raise SystemExit(f"unknown workload {name}")


def make_rhs(g, wl, torch, synth, dev):
    x1, x2, x3 = (torch.tensor(c, dtype=torch.float64, device=dev) for c in g.grid_coords())
    k, a = synth.sine_modes(wl["seed"])
    u, f = synth.sine_solution(k, a, (1.0, 1.0, 1.0), x1[None, None, :], x2[None, :, None],
                               x3[:, None, None], wl["lam"], xp=torch)
    return u.contiguous(), f.contiguous()


def smoother_flops(n, p):
    """Algorithmic flops of one smoother application: 37 n_S^3 per star.

    Stars are all vertices of the mesh except the 8 domain corners, whose
    three planes are Dirichlet (Alg. 1, op count of Sec. 3.2).
    """
    nS = 2 * p - 1
    nstars = (n[0] + 1) * (n[1] + 1) * (n[2] + 1) - 8
    return 37.0 * nS ** 3 * nstars


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


def time_smoother(g, torch, dev, dtype, reps=50):
    """Average duration of one smoothing update u += S(r) on the finest
    level, HIP events recorded on the stream the kernel is launched on."""
    import paper_1808_03595_amd as pmg
    L = g.num_levels()
    n = g.skeleton_len(L)
    tdt = torch.float64 if dtype == pmg.F64 else torch.float32
    r = torch.randn(n, dtype=tdt, device=dev)
    tmp = torch.empty(g.grid_shape(), dtype=torch.float64, device=dev)
    g.skeleton_to_grid(r, tmp, dtype)       # zero the unused slots of r
    g.grid_to_skeleton(tmp, r, dtype)
    u = torch.zeros_like(r)
    s = torch.cuda.current_stream()
    for _ in range(3):
        g.schwarz_smooth_add(L, r, u, 1.0, dtype, stream=s)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        g.schwarz_smooth_add(L, r, u, 1.0, dtype, stream=s)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def cpu_baseline(wl, coarse_rtol):
    """The FP64 oracle's complete solve of the workload (condensation, ipCG
    to 1e-10 with the same coarse tolerance, recovery) on the host cores."""
    import numpy as np
    import synth
    from oracle import mesh as omesh, solver
    threads = len(os.sched_getaffinity(0))
    n = wl["n"]
    o = omesh.Mesh.box(n, wl["p"], wl["lam"], wl["alpha"])
    X3, X2, X1 = o.coords()
    k, a = synth.sine_modes(wl["seed"])
    _, f = synth.sine_solution(k, a, (1.0, 1.0, 1.0), X1, X2, X3, wl["lam"])
    f = np.broadcast_to(f, o.shape).copy()
    t0 = time.perf_counter()
    res = solver.solve(o, f, method="kMG", rtol=1e-10, coarse_rtol=coarse_rtol, coarse_maxit=2000)
    return dict(t=time.perf_counter() - t0, iters=res.iters, threads=threads)


def coarse_levels(p, alpha, ne):
    """Degree-1 levels below p_0 = 2 (Sec. 4.2's low-order coarse grid) for
    degree p, stretching alpha and ne elements.

    Measured on one MI355X (whole solves to 1e-10): at p <= 4 the coarse
    problem is most of the mesh and six levels win.  At p = 8 one level wins
    on uniform meshes of 16^3 elements or more (the paper's test problem at
    16^3..40^3 elements: 1.2-2.1x; the p = 8 sweep point: 1.28x) and loses on
    8^3 elements and on the stretched default workload (aspect ratio 8: 7 ->
    10 outer iterations).  At p >= 12 (meshes of 18^3 elements or fewer in
    the sweep, deeper p-hierarchies) it loses 0-25 %.
    """
    if p <= 4:
        return 6
    return 1 if (p <= 8 and alpha == 1.0 and ne >= 16 ** 3) else 0


def learned_damping(wl, L):
    """omega predicted by the trained network for this mesh, or None."""
    import synth
    from paper_1808_03595_amd.learn import DampingMLP, predict_damping
    model = DampingMLP.load()
    if model is None:
        return None
    n = wl["n"]
    hs = [synth.stretched_widths(n[d], wl["alpha"]) for d in range(3)]
    return predict_damping(model, wl["p"], wl["lam"], hs[0], hs[1], hs[2], L)


SWEEP = (2, 4, 8, 12, 16, 24, 32, 48)


def p_sweep(torch, pmg, synth, dev, coarse_rtol, steps):
    """Unknowns/s versus p at about 1e7 unknowns (n = round(215.44 / p)
    elements per direction, uniform, lambda = 1, 8 sine modes), plain FP64
    and mixed precision with the learned damping, one whole solve each after
    one warm-up."""
    out = []
    for p in SWEEP:
        nn = int(round(215.44 / p))
        wl = dict(n=(nn, nn, nn), p=p, lam=1.0, alpha=1.0, seed=0)
        g = pmg.create_mesh(nn, nn, nn, p, 1.0, 1.0)
        g.set_cycle(0, coarse_rtol, 5000)
        # the CG on the coarse problem grows like n_e^(4/3) (Sec. 4.2), so
        # degree-1 levels go below it
        hmg = coarse_levels(p, 1.0, nn ** 3)
        if hmg:
            g.set_coarse_mg(hmg, 0.8, 2)
        L = g.num_levels()
        u_ex, f = make_rhs(g, wl, torch, synth, dev)
        u = torch.zeros_like(f)
        ndof = nn ** 3 * p ** 3
        row = {"p": p, "n": nn, "ndof": ndof, "levels": L + 1,
               "coarse": f"{hmg} degree-1 levels + CG" if hmg else "CG on p_0 = 2"}
        omega = learned_damping(wl, L) if L > 0 else None
        for name, dtype, om in (("fp64", pmg.F64, None), ("mixed_learned", pmg.F32, omega)):
            g.set_damping(om)
            g.pcg_solve(f, u, 1e-10, 300, dtype)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                st = g.pcg_solve(f, u, 1e-10, 300, dtype)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            err = (torch.linalg.vector_norm(u - u_ex) / torch.linalg.vector_norm(u_ex)).item()
            row[name] = {"unknowns_per_s": ndof / dt, "ms": dt * 1e3, "iters": st.iters,
                         "rel_res": st.rel_res, "rel_err_vs_exact": err, "status": st.status}
        log(f"[bench] sweep p={p} n={nn}: fp64 {row['fp64']['ms']:.1f} ms ({row['fp64']['iters']} it), "
            f"mixed+learned {row['mixed_learned']['ms']:.1f} ms ({row['mixed_learned']['iters']} it)")
        out.append(row)
        g.close()
        del u, f, u_ex
        torch.cuda.empty_cache()
    return out


NSWEEP = (8, 16, 24, 32, 40)


def n_sweep(torch, pmg, synth, dev, coarse_rtol, steps):
    """Runtime versus the number of unknowns (the linear-scaling claim,
    Sec. 5.2): the paper's runtime test problem on (0, 2 pi)^3 (manufactured
    solution with k = 5, lambda = 0, its values as inhomogeneous Dirichlet
    data on the whole boundary), p = 8 on n^3 uniform elements, plain FP64
    and mixed precision with the learned damping, one whole solve each after
    one warm-up."""
    out = []
    p = 8
    for nn in NSWEEP:
        h = [2.0 * math.pi / nn] * nn
        g = pmg.create_mesh_widths(h, h, h, p, 0.0)
        g.set_cycle(0, coarse_rtol, 5000)
        hmg = coarse_levels(p, 1.0, nn ** 3)
        g.set_coarse_mg(hmg, 0.8, 2)
        L = g.num_levels()
        x1, x2, x3 = (torch.tensor(c, dtype=torch.float64, device=dev) for c in g.grid_coords())
        u_ex, f = synth.paper_test_solution(5.0, 0.0, x1[None, None, :], x2[None, :, None],
                                            x3[:, None, None], xp=torch)
        u_ex, f = u_ex.contiguous(), f.contiguous()
        u = torch.zeros_like(f)
        ndof = nn ** 3 * p ** 3
        row = {"n": nn, "p": p, "ndof": ndof,
               "coarse": f"{hmg} degree-1 level(s) + CG" if hmg else "CG on p_0 = 2"}
        omega = learned_damping(dict(n=(nn, nn, nn), p=p, lam=0.0, alpha=1.0), L)
        for name, dtype, om in (("fp64", pmg.F64, None), ("mixed_learned", pmg.F32, omega)):
            g.set_damping(om)
            g.pcg_solve_dirichlet(f, u_ex, u, 1e-10, 300, dtype)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                st = g.pcg_solve_dirichlet(f, u_ex, u, 1e-10, 300, dtype)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            err = (u - u_ex).abs().max().item()
            row[name] = {"ms": dt * 1e3, "iters": st.iters, "ns_per_unknown": dt * 1e9 / ndof,
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2a")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--coarse-rtol", type=float, default=3e-2,
                    help="relative tolerance of the coarse CG (the paper leaves it open)")
    ap.add_argument("--damping", choices=["learned", "one"], default="learned")
    ap.add_argument("--hmg-levels", type=int, default=None,
                    help="degree-1 levels below p_0 (0: the paper's CG on p_0 = 2; "
                         "default: 6 at p <= 4; 1 at p <= 8 on uniform meshes of >= 16^3 elements; else 0)")
    ap.add_argument("--hmg-omega", type=float, default=0.8)
    ap.add_argument("--hmg-nu", type=int, default=2)
    ap.add_argument("--kernel-only", action="store_true",
                    help="run only the smoother timing loop (for counter profiles)")
    ap.add_argument("--copy-only", action="store_true",
                    help="run one 512 MiB device copy (scale of the byte counters)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the p sweep at 1e7 unknowns")
    ap.add_argument("--no-nsweep", action="store_true",
                    help="skip the sweep over the unknown count (the paper's test problem, p = 8)")
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
    wl = workload(args.workload)
    n, p = wl["n"], wl["p"]
    g = pmg.create_mesh(n[0], n[1], n[2], p, wl["lam"], wl["alpha"])
    L = g.num_levels()
    if args.kernel_only:
        t = time_smoother(g, torch, dev, pmg.F32, reps=100)
        log(f"[bench] {ROOFLINE_KERNEL}: {t * 1e6:.2f} us per launch")
        return
    g.set_cycle(0, args.coarse_rtol, 2000)
    hmg = args.hmg_levels if args.hmg_levels is not None else coarse_levels(p, wl["alpha"], n[0] * n[1] * n[2])
    if hmg:
        g.set_coarse_mg(hmg, args.hmg_omega, args.hmg_nu)
    u_ex, f = make_rhs(g, wl, torch, synth, dev)
    u = torch.zeros_like(f)
    ndof = n[0] * n[1] * n[2] * p ** 3

    def run(dtype, omega, steps, warm):
        g.set_damping(omega)
        for _ in range(warm):
            g.pcg_solve(f, u, 1e-10, 200, dtype)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = None
        for _ in range(steps):
            st = g.pcg_solve(f, u, 1e-10, 200, dtype)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = (torch.linalg.vector_norm(u - u_ex) / torch.linalg.vector_norm(u_ex)).item()
        return dt / steps, st, err

    omega = learned_damping(wl, L) if args.damping == "learned" else None
    log(f"[bench] workload {args.workload}: n={n} p={p} ndof={ndof} omega={omega}")
    t64, st64, err64 = run(pmg.F64, None, args.steps, args.warmup)
    log(f"[bench] fp64: {t64*1e3:.2f} ms/solve iters={st64.iters} rel_res={st64.rel_res:.2e} "
        f"coarse_iters={st64.coarse_iters} err_vs_exact={err64:.2e}")
    t1, st1, err1 = run(pmg.F32, None, args.steps, args.warmup)
    log(f"[bench] mixed omega=1: {t1*1e3:.2f} ms/solve iters={st1.iters} rel_res={st1.rel_res:.2e} "
        f"coarse_iters={st1.coarse_iters} err_vs_exact={err1:.2e}")
    if omega is not None:
        t32, st32, err32 = run(pmg.F32, omega, args.steps, args.warmup)
        log(f"[bench] mixed learned: {t32*1e3:.2f} ms/solve iters={st32.iters} rel_res={st32.rel_res:.2e} "
            f"coarse_iters={st32.coarse_iters} err_vs_exact={err32:.2e}")
    else:
        t32, st32, err32 = t1, st1, err1
    g.set_damping(None)

    roof = None
    if L > 0:   # p_0 = 2 alone has no smoothed level
        ts64 = time_smoother(g, torch, dev, pmg.F64)
        ts32 = time_smoother(g, torch, dev, pmg.F32)
        fl = smoother_flops(n, p)
        ach32 = fl / ts32 / 1e12
        ach64 = fl / ts64 / 1e12
        log(f"[bench] smoother f64 {ts64*1e6:.1f} us ({ach64:.2f} TF/s), f32 {ts32*1e6:.1f} us ({ach32:.2f} TF/s)")
        traffic = None
        if TRAFFIC["kernels_sha1"] == kernels_sha1() and args.workload == "c2a":
            traffic = TRAFFIC["bytes_per_launch"]
        roof = {"bound": "mfma", "kernel": smoother_kernel(p, "float"),
                "achieved": ach32, "peak": PEAK["f32"], "unit": "TFLOP/s",
                "frac": ach32 / PEAK["f32"], "traffic": traffic,
                "us_per_launch": ts32 * 1e6,
                "fp64": {"kernel": smoother_kernel(p, "double"), "achieved": ach64, "peak": PEAK["f64"],
                         "frac": ach64 / PEAK["f64"], "us_per_launch": ts64 * 1e6}}

    cpu = None
    if not args.no_cpu:
        c = cpu_baseline(wl, args.coarse_rtol)
        cpu = {"value": ndof / c["t"], "unit": "unknowns/s", "cores": c["threads"], "kind": "oracle",
               "sample": (f"the FP64 oracle's complete solve of the same workload ({c['iters']} ipCG "
                          f"iterations to 1e-10, coarse CG to {args.coarse_rtol:g}), timed once: {c['t']:.1f} s")}
        log(f"[bench] cpu oracle: {c['t']:.2f} s, {c['iters']} iterations")

    sweep = None
    if not args.no_sweep:
        g.close()
        sweep = p_sweep(torch, pmg, synth, dev, args.coarse_rtol, 1)
    nsweep = None
    if not args.no_nsweep and not args.no_sweep:
        nsweep = n_sweep(torch, pmg, synth, dev, args.coarse_rtol, 1)

    line = {
        "metric": "solved unknowns/s to 1e-10 residual vs p; FP32-MG+learned vs plain FP64",
        "value": ndof / t32,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-vcycle/f64-cg",
        "data": "synthetic",
        "config": {"workload": f"{n[0]}x{n[1]}x{n[2]} elements, p={p}, lambda={wl['lam']:g}, "
                               f"stretch alpha={wl['alpha']:.4f} (AR {wl['alpha']**(n[0]-1):.1f}), "
                               f"8 sine modes seed {wl['seed']}",
                   "ndof": ndof, "iters": st32.iters, "rel_res": st32.rel_res,
                   "damping": "learned" if omega is not None else "omega=1 (paper)",
                   "omega": omega,
                   "coarse": (f"Jacobi CG on p_0=2 to rel. {args.coarse_rtol:g}" if not hmg else
                              f"{hmg} degree-1 levels + CG"),
                   "coarse_iters_per_solve": st32.coarse_iters,
                   "mixed_omega1_unknowns_per_s": ndof / t1, "mixed_omega1_iters": st1.iters,
                   "fp64_unknowns_per_s": ndof / t64, "fp64_iters": st64.iters,
                   "fp64_ms_per_solve": t64 * 1e3,
                   "rel_err_vs_exact_mixed": err32, "rel_err_vs_exact_fp64": err64},
        "roofline": roof,
        "cpu_baseline": cpu,
        "p_sweep": sweep,
        "n_sweep": nsweep,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
