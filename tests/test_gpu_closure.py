"""Closure features, targets and the one-point closure step on the GPU,
through the C ABI, against the FP64 oracle and its feature reference."""
import math

import numpy as np
import pytest

from paper_1502_01159_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01159_amd import pibm

    pibm.lib()
    return pibm


def sub_grid(P, R=0.6):
    """One-point particles must be sub-grid (the paper's d <= h): with the
    weight pi d^2 / 4 of a larger body the explicit exchange over-corrects
    the fluid several times over and diverges.  They are held fixed: a
    sub-grid body lighter than its exchange weight is unstable under the
    explicit coupling (added mass), and the flow here comes from their heat."""
    P = np.array(P, dtype=float)
    P[:, 9] = R
    P[:, 12] = W.FIXED
    return P


def reference(oracle_mod, ref, cfg):
    from oracle import closure_oracle as C

    d = oracle_mod.derive(cfg)
    rho, j, S = ref.raw_moments()
    ref.exchange()
    q, r = ref.particles(), ref.reactions()
    shape = (cfg.get("nz", 1) if cfg["dim"] == 3 else 1, cfg["ny"], cfg["nx"])
    X, s, Tf = C.features(rho, j, S, shape, cfg["periodic"], q, d["nu"], d["gbeta"], cfg["dim"])
    T = C.targets(r[:, :3], r[:, 6], s, q[:, 12], q[:, 14] - Tf, d["nu"], d["alpha"], cfg["dim"])
    return X, T, s, d, Tf


def coarse_array():
    """150 fixed spheres of D = 8 in a periodic 96^3 box, coarsened 4x: points
    of D = 2 on a 24^3 lattice, cells of width 3 (8 per axis), so the
    neighbour search covers part of the box: the 4 nearest of most particles
    lie within two cell widths, those of the rest do not."""
    from paper_1502_01159_amd import closure as CL

    cfg, P = CL.fixed_array(L=96, n=150, D=8.0, seed=21)
    return CL.coarsen(cfg, P, c=4)


def nearest_within_cells(P, cfg, nn=4, width=3.0):
    """Per particle: whether its nn-th nearest centre (minimum image) lies
    within two cell widths."""
    L = np.array([cfg["nx"], cfg["ny"], cfg["nz"]], dtype=float)
    x = P[:, 0:3]
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    return np.sort(r, axis=1)[:, nn - 1] < 2 * width


@pytest.mark.parametrize("name,mode", [("c3_small", 1), ("c2_small", 1), ("c3_small", 2), ("coarse_array", 2)])
def test_features_and_targets_match_oracle(gpu, oracle_mod, name, mode):
    if name == "coarse_array":
        cfg, P = coarse_array()
        inside = nearest_within_cells(P, cfg)
        assert inside.any() and not inside.all()   # both branches of the search are taken
        steps = 8
    else:
        cfg, P = W.workload(name)
        steps = 40
    cfg = W.with_overrides(cfg, marker_mode=mode)
    if mode == 2 and name != "coarse_array":
        P = sub_grid(P)
    sim = gpu.Simulation(cfg, P, storage="f64")
    ref = oracle_mod.Oracle(cfg, P)
    sim.step(steps)
    ref.step(steps)
    x, t = sim.features()
    X, T, _, _, _ = reference(oracle_mod, ref, cfg)
    # FP64 on both sides, FP32 on output
    for col in range(16):
        sc = max(1.0, np.abs(X[:, col]).max())
        assert np.abs(x[:, col] - X[:, col]).max() <= 2e-6 * sc, col
    for col in range(4):
        sc = max(1e-3, np.abs(T[:, col]).max())
        assert np.abs(t[:, col] - T[:, col]).max() <= 2e-6 * sc, col
    # the call did not advance the state
    x2, t2 = sim.features()
    assert np.array_equal(x, x2) and np.array_equal(t, t2)
    sim.close()


def test_closure_step_applies_network_outputs(gpu, oracle_mod):
    """One step with the network as the closure: the particles' reactions are
    the denormalised outputs for the features of the state the step starts
    from, turned out of the slip frame (force) and scaled (heat), with no
    fluid torque."""
    import torch
    from oracle import mlp_oracle as M

    cfg, P = W.workload("c3_small")
    cfg = W.with_overrides(cfg, marker_mode=2)
    P = sub_grid(P)
    sim = gpu.Simulation(cfg, P, storage="f64")
    ref = oracle_mod.Oracle(cfg, P)
    sim.step(20)
    ref.step(20)
    mlp = gpu.Mlp(seed=5, max_batch=64)
    x, _ = sim.features()
    mu = x.mean(0).astype(np.float32)
    sd = (x.std(0) + 0.1).astype(np.float32)
    norm = np.concatenate([mu, sd, np.array([0.5, -0.2, 0.1, 0.3], np.float32), np.array([2.0, 1.0, 1.5, 0.5], np.float32)])
    sim.set_closure(mlp, norm)
    _, _, s, d, Tf = reference(oracle_mod, ref, cfg)
    xn = torch.tensor((x - mu) / sd, dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()
    y = mlp.forward(xn).cpu().numpy().astype(np.float64) * norm[36:40] + norm[32:36]
    sim.step(1)
    _, fth = sim.particles()
    from oracle import closure_oracle as C
    for p in range(len(P)):
        e1, e2, e3 = C.slip_frame(s[p], 3)
        fs = 3 * math.pi * d["nu"] * 2 * P[p, 9] * np.linalg.norm(s[p])
        F = (y[p, 0] * e1 + y[p, 1] * e2 + y[p, 2] * e3) * fs
        H = y[p, 3] * math.pi * 2 * P[p, 9] * d["alpha"] * (P[p, 11] - Tf[p])
        sc = np.abs(F).max() + 1e-12
        assert np.abs(fth[p, :3] - F).max() <= 2e-2 * sc, p
        assert fth[p, 6] == pytest.approx(H, rel=2e-2, abs=1e-9)
        assert not fth[p, 3:6].any()
    sim.set_closure(None)
    mlp.close()
    sim.close()


def test_closure_two_streams_match_one_stream(gpu):
    """With the network as the closure, binning on a second stream beside the
    closure's kernels and the DEM beside the lattice give the same bits as one
    stream."""
    cfg, P = W.workload("c3_small")
    cfg = W.with_overrides(cfg, marker_mode=2)
    P = sub_grid(P)
    mlp = gpu.Mlp(seed=5, max_batch=64)
    probe = gpu.Simulation(cfg, P, storage="f32")
    x, _ = probe.features()
    probe.close()
    mu = x.mean(0).astype(np.float32)
    sd = (x.std(0) + 0.1).astype(np.float32)
    norm = np.concatenate([mu, sd, np.array([0.5, -0.2, 0.1, 0.3], np.float32), np.array([2.0, 1.0, 1.5, 0.5], np.float32)])
    out = []
    for streams in (1, 2):
        sim = gpu.Simulation(dict(cfg, streams=streams), P, storage="f32")
        sim.set_closure(mlp, norm)
        sim.step(5)
        assert sim.sync() == gpu.OK
        f, g = sim.populations()
        q, r = sim.particles()
        out.append((f, g, q, r))
        sim.set_closure(None)
        sim.close()
    mlp.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_learned_closure_beats_point_exchange(gpu):
    """What the network gains over the method without it.  Resolved runs of
    fixed hot spheres in a driven periodic box give samples; the network is
    trained on the GPU; then the same problem on a 4x coarser lattice runs
    with one point per sphere, once with the paper's point exchange and once
    with the learned closure.  Per-sphere force and heat at matching physical
    times, against a resolved run of an arrangement not trained on: the
    learned closure's errors are the smaller ones, and on held-out samples
    the network reproduces force and Nusselt number."""
    import torch
    from paper_1502_01159_amd import closure as CL

    Xs, Ts, Is = [], [], []
    for seed, n in ((21, 120), (22, 180), (23, 240)):
        cfg, P = CL.fixed_array(n=n, seed=seed)
        X, T, ids, _ = CL.harvest(gpu, cfg, P, steps=1600, every=100, start=200)
        Xs.append(X); Ts.append(T); Is.append(ids + 1000 * seed)
    X, T, I = np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Is)
    ok = CL.usable(X)
    X, T, I = X[ok], T[ok], I[ok]
    hold = (I % 10) == 0
    norm = CL.norm_stats(X[~hold], T[~hold])
    mlp = gpu.Mlp(seed=7, max_batch=4096)
    hist = CL.train(torch, mlp, X[~hold], T[~hold], norm, epochs=60, batch=1024, lr=1e-3)
    assert hist[-1] < 0.3 * hist[0]
    Y = CL.predict(torch, mlp, X[hold], norm)
    assert CL.rel_l2(Y[:, :3], T[hold][:, :3]) < 0.25
    assert CL.rel_l2(Y[:, 3], T[hold][:, 3]) < 0.15

    cfg, P = CL.fixed_array(n=180, seed=31)
    times = [400, 800, 1200, 1600]
    res = CL.run_states(gpu, cfg, P, times)
    cc, Pc = CL.coarsen(cfg, P)
    tc = [t // 16 for t in times]
    pt = CL.run_states(gpu, cc, Pc, tc)
    ml = CL.run_states(gpu, cc, Pc, tc, mlp=mlp, norm=norm)
    eF_pt = np.mean([CL.rel_l2(pt[c][0], res[f][0]) for f, c in zip(times, tc)])
    eF_ml = np.mean([CL.rel_l2(ml[c][0], res[f][0]) for f, c in zip(times, tc)])
    eH_pt = np.mean([CL.rel_l2(4 * pt[c][1], res[f][1]) for f, c in zip(times, tc)])
    eH_ml = np.mean([CL.rel_l2(4 * ml[c][1], res[f][1]) for f, c in zip(times, tc)])
    print(f"coarse vs resolved, mean over times: force {eF_pt:.3f} (point) {eF_ml:.3f} (network); "
          f"heat {eH_pt:.3f} (point) {eH_ml:.3f} (network)")
    assert eF_ml < eF_pt and eH_ml < eH_pt
    mlp.close()
