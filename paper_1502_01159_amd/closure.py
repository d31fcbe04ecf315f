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


def force_space_errors(Y, T, X):
    """Relative L2 errors of predicted targets Y against T weighted back to
    physical size: the force components times the slip (Re_p, column 0 of the
    features), the Nusselt number times T_p - T_f (column 3).  Unlike errors
    of the normalised targets, these are not dominated by samples with a
    vanishing slip or temperature difference."""
    eF = rel_l2(Y[:, :3] * X[:, :1], T[:, :3] * X[:, :1])
    eH = rel_l2(Y[:, 3] * X[:, 3], T[:, 3] * X[:, 3])
    return eF, eH


def sedimentation_study(pibm, torch, steps=3800, every=20, start=500, epochs=60, re_min=0.05, coarse_steps=200,
                        log=print):
    """The closure at the scale of the 3D sedimentation case: samples every
    `every` steps after `start` from the full 256 x 256 x 512 case with 2000
    spheres at Gr = 0, 100 and 1000 (about 10^6), 10% of the particles held
    out by id, GPU training, learning curves of the held-out and training
    errors in force space, then the 4x coarser case (one point per sphere) with
    the network, with the network and its fallback to the point exchange
    outside the central 99% of each training feature, and with the paper's
    point exchange alone, reporting the largest particle speed, the watchdog
    status and the share of particles on the network as the coarse runs
    advance."""
    Xs, Ts, Is, Gs = [], [], [], []
    for k, gr in enumerate((0, 100, 1000)):
        cfg, P = W.workload(f"c3_gr{gr}")
        X, T, ids, _ = harvest(pibm, cfg, P, steps=steps, every=every, start=start)
        Xs.append(X); Ts.append(T); Is.append(ids + 10000 * k); Gs.append(np.full(len(X), gr))
    X, T, I, G = map(np.concatenate, (Xs, Ts, Is, Gs))
    ok = (X[:, 0] > re_min) & (np.abs(X[:, 3]) > 1e-3)
    log(f"samples {len(X)}, usable {int(ok.sum())} (Re_p > {re_min}, |T_p - T_f| > 1e-3)")
    X, T, I, G = X[ok], T[ok], I[ok], G[ok]
    hold = (I % 10) == 0
    norm = norm_stats(X[~hold], T[~hold])
    mlp = pibm.Mlp(seed=7, max_batch=4096)
    curve = []
    for e0 in range(0, epochs, 5):
        lr = 1e-3 if e0 < 2 * epochs // 3 else 3e-4
        hist = train(torch, mlp, X[~hold], T[~hold], norm, epochs=5, batch=4096, lr=lr, seed=e0)
        hF, hH = force_space_errors(predict(torch, mlp, X[hold], norm), T[hold], X[hold])
        sub = np.nonzero(~hold)[0][:200000]
        tF, tH = force_space_errors(predict(torch, mlp, X[sub], norm), T[sub], X[sub])
        curve.append((e0 + 5, hist[-1], hF, hH, tF, tH))
        log(f"epoch {e0 + 5}: loss {hist[-1]:.4f}  held-out force {hF:.3f} heat {hH:.3f}  "
            f"training force {tF:.3f} heat {tH:.3f}")
    per_gr = {}
    for gr in (0, 100, 1000):
        m = hold & (G == gr)
        per_gr[gr] = force_space_errors(predict(torch, mlp, X[m], norm), T[m], X[m])
        log(f"Gr {gr}: held-out force {per_gr[gr][0]:.3f} heat {per_gr[gr][1]:.3f}")
    # the network is trusted on the central 99% of each training feature;
    # outside it a particle falls back to the point exchange
    lo = np.quantile(X[~hold], 0.005, axis=0).astype(np.float32)
    hi = np.quantile(X[~hold], 0.995, axis=0).astype(np.float32)
    cfg, P = W.workload("c3_gr100")
    cc, Pc = coarsen(cfg, P)
    coarse = {}
    for mode in ("network", "network with fallback", "point exchange"):
        sim = pibm.Simulation(cc, Pc, storage="f32")
        if mode != "point exchange":
            sim.set_closure(mlp, norm)
        if mode == "network with fallback":
            sim.set_closure_range(lo, hi)
        trace = []
        for k in range(0, coarse_steps, 10):
            sim.step(10)
            st = sim.sync()
            q, _ = sim.particles(check=False)
            frac = float("nan")
            if st == pibm.OK and mode == "network with fallback":
                x, _ = sim.features()
                frac = float(np.mean(np.all((x >= lo) & (x <= hi), axis=1)))
            trace.append((k + 10, st, float(np.abs(q[:, 3:6]).max()), frac))
            if st != pibm.OK:
                break
        log(f"coarse {mode}: " + ", ".join(
            f"step {a}: max|U_p| {c:.3f}" + ("" if b == pibm.OK else " (watchdog)") +
            ("" if np.isnan(d) else f" on network {d:.2f}")
            for a, b, c, d in trace[::4] + ([trace[-1]] if len(trace) % 4 != 1 else [])))
        coarse[mode] = trace
        sim.set_closure(None)
        sim.close()
    mlp.close()
    return dict(curve=curve, per_gr=per_gr, coarse=coarse, range=(lo, hi))


if __name__ == "__main__":
    import torch

    from . import pibm

    sedimentation_study(pibm, torch)

