"""Learned per-level damping of the Schwarz smoother.

The V-cycle updates u_l += omega_l Smoother_l(r_l); the paper uses
omega_l = 1.  Here a small FP32 network predicts omega_l for the finest
NOUT levels from (p, lambda h_min^2, aspect ratio).  Training data come from
the solver itself: for each sample mesh the deployed solver (mixed-precision
Krylov-accelerated MG, Alg. 5) is run for a few iterations and its
convergence factor rho = (|r_n| / |r_0|)^(1/n) (Sec. 5.2) is measured on a
grid of damping values, level by level from the finest one (coordinate
search).  The network is trained on the GPU by
the library's own forward, loss, backward and Adam kernels; omega = 1
remains the fallback when no trained parameters are available.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import F32, F64, create_mesh_widths, mlp_adam, mlp_backward, mlp_forward, mlp_loss, mlp_nparams

NOUT = 4                                   # damped levels: finest four (p <= 32)
OMEGA_GRID = np.round(np.arange(0.5, 1.5001, 0.05), 2)
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "damping_mlp.npz")


def mlp_features(p, lam, hmin, ar):
    """Scaled network inputs: (p/32, log10(1 + lambda h_min^2)/4, log2(AR)/4)."""
    return np.array([p / 32.0, math.log10(1.0 + lam * hmin * hmin) / 4.0,
                     math.log2(max(ar, 1.0)) / 4.0], dtype=np.float32)


def mesh_features(p, lam, hx, hy, hz):
    """(p, lambda h_min^2, AR): h_min over all element widths, AR the largest
    element aspect ratio max(h) / min(h)."""
    hs = [np.asarray(h, dtype=np.float64) for h in (hx, hy, hz)]
    hmin = min(float(h.min()) for h in hs)
    ar = 1.0
    for a in hs[0]:
        for b in hs[1]:
            for c in hs[2]:
                ar = max(ar, max(a, b, c) / min(a, b, c))
    return mlp_features(p, lam, hmin, ar)


def glorot(nout=NOUT, seed=0):
    """Glorot-uniform initial parameters (zero biases), float32."""
    r = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((3, 64), (64, 64), (64, nout)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(r.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


class DampingMLP:
    """FP32 network 3 -> 64 -> 64 -> NOUT held in device memory."""

    def __init__(self, params=None, nout=NOUT, seed=0, trained=None):
        import torch
        self.torch = torch
        self.nout = nout
        # outputs that had training targets; the others are never used (the
        # paper's omega = 1 stands in for them)
        self.trained = np.ones(nout, dtype=bool) if trained is None else np.asarray(trained, dtype=bool)
        self.dev = torch.device("cuda:0")
        p = glorot(nout, seed) if params is None else np.asarray(params, dtype=np.float32)
        assert p.size == mlp_nparams(nout)
        self.params = torch.as_tensor(p, device=self.dev).contiguous()

    @classmethod
    def load(cls, path=DEFAULT_WEIGHTS):
        if not os.path.exists(path):
            return None
        with np.load(path, allow_pickle=False) as z:
            trained = z["trained"] if "trained" in z.files else None
            return cls(z["params"], int(z["nout"]), trained=trained)

    def save(self, path, **meta):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.savez(path, params=self.params.cpu().numpy(), nout=np.int32(self.nout),
                 trained=self.trained.astype(np.int8), meta=np.array(json.dumps(meta)))

    def predict(self, X):
        torch = self.torch
        X = torch.as_tensor(np.asarray(X, dtype=np.float32).reshape(-1, 3), device=self.dev)
        B = X.shape[0]
        y = torch.empty(B, self.nout, dtype=torch.float32, device=self.dev)
        cache = torch.empty(B, 128 + self.nout, dtype=torch.float32, device=self.dev)
        mlp_forward(self.params, X, y, cache, B, self.nout)
        return y.cpu().numpy()

    def train(self, X, T, M, steps=3000, lr=1e-3, log_every=500):
        """Full-batch Adam on the masked MSE; every step runs on the GPU."""
        torch = self.torch
        X = torch.as_tensor(np.asarray(X, dtype=np.float32), device=self.dev).contiguous()
        T = torch.as_tensor(np.asarray(T, dtype=np.float32), device=self.dev).contiguous()
        M = torch.as_tensor(np.asarray(M, dtype=np.float32), device=self.dev).contiguous()
        B, n = X.shape[0], self.params.numel()
        y = torch.empty(B, self.nout, dtype=torch.float32, device=self.dev)
        cache = torch.empty(B, 128 + self.nout, dtype=torch.float32, device=self.dev)
        dy = torch.empty_like(y)
        loss = torch.empty(1, dtype=torch.float32, device=self.dev)
        grad = torch.empty_like(self.params)
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        hist = []
        for t in range(1, steps + 1):
            mlp_forward(self.params, X, y, cache, B, self.nout)
            mlp_loss(y, T, M, dy, loss, B, self.nout)
            mlp_backward(self.params, X, cache, dy, grad, B, self.nout)
            mlp_adam(self.params, grad, m, v, n, lr, 0.9, 0.999, 1e-8, t)
            if t == 1 or t % log_every == 0 or t == steps:
                hist.append((t, float(loss.item())))
        return hist


def convergence_factor(mesh, f, omega, cycles=2):
    """rho over the first `cycles` iterations of the deployed solver
    (mixed-precision Krylov-accelerated MG, Alg. 5) with damping `omega`
    (finest first).  Two iterations keep the residual well above rounding
    level even where one iteration gains 1e-6."""
    torch = __import__("torch")
    mesh.set_damping(list(omega))
    u = torch.zeros_like(f)
    st = mesh.pcg_solve(f, u, 0.0, cycles, F32)
    h = st.history()
    if len(h) < 2 or h[0] == 0.0 or not np.isfinite(h[-1]) or h[-1] == 0.0:
        return float("inf")
    return (h[-1] / h[0]) ** (1.0 / (len(h) - 1))


def grid_search(mesh, f, L, cycles=2, grid=OMEGA_GRID, tie=0.25):
    """Coordinate search over omega, finest level first.  Among the values
    whose rho is within a factor (1 + tie) of the best, the one closest to 1
    is taken, so that only a clear gain moves a level away from the paper's
    omega = 1.  Returns (omega list of length L, rho at the result, rho at
    omega = 1)."""
    om = [1.0] * L
    rho1 = convergence_factor(mesh, f, om, cycles)
    best = rho1
    for j in range(L):
        scores = []
        for w in grid:
            trial = list(om)
            trial[j] = float(w)
            scores.append((convergence_factor(mesh, f, trial, cycles), float(w)))
        rmin = min(s[0] for s in scores)
        ok = [s for s in scores if s[0] <= rmin * (1.0 + tie)]
        rho_j, w_j = min(ok, key=lambda s: (abs(s[1] - 1.0), s[0]))
        om[j] = w_j
        best = rho_j
    mesh.set_damping(None)
    return om, best, rho1


def sample_mesh(p, lam_h2, ar, n=4):
    """Anisotropic brick mesh of Sec. 5.3 (scaled) with lambda from lambda h^2."""
    import synth
    (hx, hy, hz), _ = synth.anisotropic_widths(n, ar)
    hmin = min(hx.min(), hy.min(), hz.min())
    lam = lam_h2 / (hmin * hmin)
    return hx, hy, hz, lam


def build_dataset(degrees, lam_h2s, ars, n=4, seed=0, cycles=2, log=None):
    """Solver-measured targets for every (p, lambda h^2, AR) sample."""
    import torch
    import synth
    X, T, M, rows = [], [], [], []
    for p in degrees:
        for lh in lam_h2s:
            for ar in ars:
                hx, hy, hz, lam = sample_mesh(p, lh, ar, n)
                g = create_mesh_widths(hx, hy, hz, p, lam)
                L = g.num_levels()
                if L == 0:
                    continue
                g.set_cycle(0, 3e-2, 2000)
                f = torch.as_tensor(synth.random_grid(g.grid_shape(), seed), device="cuda:0")
                om, rho, rho1 = grid_search(g, f, min(L, NOUT), cycles)
                x = mesh_features(p, lam, hx, hy, hz)
                t = np.ones(NOUT, dtype=np.float32)
                mk = np.zeros(NOUT, dtype=np.float32)
                t[:len(om)] = om
                mk[:len(om)] = 1.0
                X.append(x)
                T.append(t)
                M.append(mk)
                rows.append(dict(p=p, lam_h2=lh, ar=ar, omega=om, rho=rho, rho_omega1=rho1))
                if log:
                    log(f"sample p={p} lam_h2={lh:g} AR={ar:g}: omega={om} rho={rho:.3e} (omega=1: {rho1:.3e})")
                g.close()
    return np.array(X), np.array(T), np.array(M), rows


def predict_damping(model, p, lam, hx, hy, hz, L):
    """omega for the finest min(L, NOUT) levels; None without a model.  A
    level whose output had no training target keeps omega = 1."""
    if model is None or L == 0:
        return None
    y = model.predict(mesh_features(p, lam, hx, hy, hz)[None, :])[0]
    return [float(v) if model.trained[j] else 1.0 for j, v in enumerate(y[:min(L, model.nout)])]
