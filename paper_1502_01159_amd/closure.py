"""Workflow of the learned closure: samples from resolved runs, training on
the GPU, and the coarse one-point runs it is judged in.

Everything numerical runs in the library's kernels (features, targets, the
network's forward/backward/Adam, the coarse steps); this module only
arranges runs and batches.

Coarsening by a factor c uses diffusive scaling: dx' = c dx, dt' = c^2 dt,
so viscosity and diffusivity keep their lattice values, velocities grow by
c, accelerations (gravity, g beta) by c^3, and forces stay the same number
in lattice units; a heat rate H shrinks by c (H / (pi D alpha) is invariant).
Node i of the fine lattice lies at (i - (c - 1)/2) / c on the coarse one.
"""
from __future__ import annotations

import math

import numpy as np

from . import workloads as W


def fixed_array(L=96, n=150, D=8.0, seed=21, nu=0.1, Pr=0.7, gbeta=2e-5, T_p=2.0):
    """Fixed hot spheres in a periodic box of side L; the fluid (T = 1,
    T_ref = 0) is driven by the uniform buoyancy g beta (T - T_ref) along +z
    and heated by the spheres (T_p), so the flow past each sphere mixes forced
    and free convection and the local temperature difference falls in time."""
    pts = W.rsa(seed, n, [D / 2] * 3, [L - D / 2] * 3, D + 1.0)
    P = np.array([W._row(c, D / 2, 1.0, T_p, W.FIXED) for c in pts])
    cfg = dict(name=f"fixed_array_{L}_{n}", dim=3, nx=L, ny=L, nz=L, periodic=[1, 1, 1], T_wall=[0.0] * 6,
               T_init=1.0, T_ref=0.0, Ra=0.0, nu=nu, Pr=Pr, Gr=0.0, Lc=D, gbeta=gbeta, gravity=0.0,
               kappa_T=1.0, marker_mode=1, marker_spacing=1.0, E_star=729.0, poisson=0.33, mu_fric=0.3,
               n_sub=1, beta_p=0.0, c_r=1.0)
    return cfg, P


def coarsen(cfg, P, c=4):
    """The same problem on a lattice c times coarser, particles as single
    points (the paper's sub-grid particles)."""
    out = dict(cfg)
    out["name"] = cfg.get("name", "case") + f"_coarse{c}"
    for k in ("nx", "ny", "nz"):
        if k in cfg:
            out[k] = max(1, cfg[k] // c) if (k != "nz" or cfg["dim"] == 3) else 1
    out["marker_mode"] = 2
    out["gbeta"] = cfg.get("gbeta", 0.0) * c ** 3
    out["gravity"] = cfg.get("gravity", 0.0) * c ** 3
    out["Lc"] = cfg.get("Lc", 1.0) / c
    Q = np.array(P, dtype=float).copy()
    dim = cfg["dim"]
    Q[:, 0:dim] = (Q[:, 0:dim] - 0.5 * (c - 1)) / c
    Q[:, 3:6] *= c
    Q[:, 6:9] *= c * c
    Q[:, 9] /= c
    return out, Q


def harvest(pibm, cfg, P, steps, every, start, storage="f32"):
    """Run a resolved simulation and collect (features, targets, particle id,
    step) every `every` steps from `start` on."""
    sim = pibm.Simulation(cfg, P, storage=storage)
    X, T, ids, when = [], [], [], []
    done = 0
    for s in range(start, steps + 1, every):
        sim.step(s - done)
        done = s
        x, t = sim.features()
        X.append(x)
        T.append(t)
        ids.append(np.arange(len(P)))
        when.append(np.full(len(P), s))
    sim.close()
    return np.concatenate(X), np.concatenate(T), np.concatenate(ids), np.concatenate(when)


def usable(X, re_min=1e-3, dT_min=1e-3):
    """Samples whose normalised targets are defined: slip and temperature
    difference not negligible."""
    return (X[:, 0] > re_min) & (np.abs(X[:, 3]) > dT_min)


def norm_stats(X, T):
    """40 floats: feature mean and std, target mean and std (std >= 1e-6)."""
    return np.concatenate([X.mean(0), np.maximum(X.std(0), 1e-6), T.mean(0), np.maximum(T.std(0), 1e-6)]).astype(np.float32)


def train(torch, mlp, X, T, norm, epochs=30, batch=4096, lr=1e-3, seed=0):
    """Adam on z-scored samples; returns the mean loss of each epoch."""
    xs = torch.tensor((X - norm[:16]) / norm[16:32], dtype=torch.float32).to(torch.bfloat16).cuda()
    ts = torch.tensor((T - norm[32:36]) / norm[36:40], dtype=torch.float32).cuda()
    n = len(X)
    rng = np.random.default_rng(seed)
    hist = []
    for _ in range(epochs):
        order = torch.tensor(rng.permutation(n), device="cuda")
        tot, nb = 0.0, 0
        for b0 in range(0, n - batch + 1 if n >= batch else 1, batch):
            idx = order[b0:b0 + batch]
            tot += mlp.train_step(xs[idx].contiguous(), ts[idx].contiguous(), lr)
            nb += 1
        hist.append(tot / max(nb, 1))
    return hist


def predict(torch, mlp, X, norm):
    xs = torch.tensor((X - norm[:16]) / norm[16:32], dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()
    y = mlp.forward(xs).cpu().numpy().astype(np.float64)
    return y * norm[36:40] + norm[32:36]


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_states(pibm, cfg, P, times, storage="f32", mlp=None, norm=None):
    """Reactions F (n, 3) and H (n) of the states at the given step counts;
    with `mlp`, the learned closure (one-point mode) acts."""
    sim = pibm.Simulation(cfg, P, storage=storage)
    if mlp is not None:
        sim.set_closure(mlp, norm)
    out = {}
    done = 0
    for s in times:
        sim.step(s - done)
        done = s
        _, fth = sim.particles()
        out[s] = (fth[:, 0:3].copy(), fth[:, 6].copy())
    if mlp is not None:
        sim.set_closure(None)
    sim.close()
    return out
