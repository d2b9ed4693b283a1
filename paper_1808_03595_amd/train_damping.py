"""Train the damping MLP on solver-measured convergence factors (GPU).

python -m paper_1808_03595_amd.train_damping [--out PATH] [--report PATH]

1. Training set: anisotropic brick meshes of 6^3 elements (Sec. 5.3 recipe,
   scaled) over p in {3, 4, 6, 8, 12, 16, 24, 32} (so that all four outputs,
   the finest four smoothed levels, get targets), lambda h^2 in {0, 1e-2, 1,
   1e2, 1e4}, AR in {1, 2, 4, 8, 16}; targets = per-level argmin of the
   convergence factor of the deployed solver (first two iterations) over
   omega in 0.5 .. 1.5 (step 0.05); values within 25 % of the best count as
   ties, which go to the value closest to 1.
2. Training: full-batch Adam (lr 1e-3) on the masked MSE, GPU kernels only.
3. Held-out evaluation: 24^3 elements, p = 12, AR in {3, 6, 12},
   lambda h^2 in {0.3, 30, 3e3}; iterations and time to a 1e-10 relative
   residual of the mixed-precision Krylov-accelerated MG with the learned
   omega versus omega = 1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(msg):
    print(msg, flush=True)


def evaluate(model, ns=24, p=12, ars=(3.0, 6.0, 12.0), lam_h2s=(0.3, 30.0, 3e3), seed=0,
             coarse_rtol=3e-2):
    import torch
    import synth
    from . import F32, create_mesh_widths
    from .learn import predict_damping, sample_mesh
    out = []
    for ar in ars:
        for lh in lam_h2s:
            hx, hy, hz, lam = sample_mesh(p, lh, ar, ns)
            g = create_mesh_widths(hx, hy, hz, p, lam)
            g.set_cycle(0, coarse_rtol, 2000)
            L = g.num_levels()
            _, lengths = synth.anisotropic_widths(ns, ar)
            x1, x2, x3 = (torch.tensor(c, dtype=torch.float64, device="cuda:0") for c in g.grid_coords())
            k, a = synth.sine_modes(seed)
            _, f = synth.sine_solution(k, a, lengths, x1[None, None, :], x2[None, :, None],
                                       x3[:, None, None], lam, xp=torch)
            f = f.contiguous()
            res = {"ar": ar, "lam_h2": lh}
            for name, om in (("omega1", None), ("learned", predict_damping(model, p, lam, hx, hy, hz, L))):
                g.set_damping(om)
                u = torch.zeros_like(f)
                g.pcg_solve(f, u, 1e-10, 300, F32)          # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = g.pcg_solve(f, u, 1e-10, 300, F32)
                torch.cuda.synchronize()
                res[name] = {"iters": st.iters, "rel_res": st.rel_res, "status": st.status,
                             "ms": (time.perf_counter() - t0) * 1e3, "omega": om}
            log(f"eval AR={ar:g} lam_h2={lh:g}: omega=1 {res['omega1']['iters']} it "
                f"{res['omega1']['ms']:.1f} ms | learned {res['learned']['omega']} "
                f"{res['learned']['iters']} it {res['learned']['ms']:.1f} ms")
            out.append(res)
            g.close()
    return out


def main():
    from .learn import DEFAULT_WEIGHTS, DampingMLP, build_dataset
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--degrees", default="3,4,6,8,12,16,24,32")
    ap.add_argument("--n", type=int, default=6, help="elements per direction of the training meshes")
    ap.add_argument("--skip-eval", action="store_true")
    args = ap.parse_args()
    degrees = [int(v) for v in args.degrees.split(",")]
    t0 = time.perf_counter()
    X, T, M, rows = build_dataset(degrees, [0.0, 1e-2, 1.0, 1e2, 1e4], [1.0, 2.0, 4.0, 8.0, 16.0], n=args.n,
                                  log=log)
    t_data = time.perf_counter() - t0
    log(f"dataset: {len(X)} samples in {t_data:.1f} s")
    model = DampingMLP(seed=0, trained=np.asarray(M).any(axis=0))
    t0 = time.perf_counter()
    hist = model.train(X, T, M, steps=args.steps, lr=1e-3)
    t_train = time.perf_counter() - t0
    log(f"training: {hist} ({t_train:.1f} s)")
    model.save(args.out, samples=len(X), steps=args.steps, final_loss=hist[-1][1])
    pred = model.predict(X)
    fit = float(np.sqrt(np.sum(M * (pred - T) ** 2) / np.sum(M)))
    log(f"saved {args.out}; rms fit error on the training targets {fit:.3f}")
    ev = [] if args.skip_eval else evaluate(model)
    if args.report:
        os.makedirs(os.path.dirname(args.report) or ".", exist_ok=True)
        with open(args.report, "w") as fh:
            json.dump({"dataset": rows, "train_loss": hist, "fit_rms": fit, "t_data_s": t_data,
                       "t_train_s": t_train, "eval": ev}, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
