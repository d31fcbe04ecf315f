#!/usr/bin/env python3
"""Throughput of the coupled thermal LBM-PIBM-DEM step on one MI355X.

One step = the whole hot path on one batch of synthetic input: Lagrangian
points (interpolation, exchange, per-particle reactions), particle->tile
binning, the fused stream/spreading/collision kernel for f and g, the DEM
neighbour lists and sub-steps, and the thermosensitive update.

Default workload: 3D sedimentation of heated spheres, 256 x 256 x 512 lattice
(D3Q19 + D3Q7), 2000 spheres of diameter 12, FP32 storage.  Prints ONE JSON
line with the MLUPS, the roofline of the dominant kernel (measured live with
HIP events on the library's stream), FP16/BF16 storage variants, and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
METRIC = "MLUPS (coupled flow+thermal+PIBM), % HBM roofline; FP32 vs FP16-storage vs MLP"
WORKLOAD_TEXT = {
    "c2": "2D sedimentation of hot disks: D2Q9+D2Q5, 512x1024, 100 disks D=20, Gr=500",
    "c3": "3D sedimentation of heated spheres: D3Q19+D3Q7, 256x256x512, 2000 spheres D=12, Gr=100",
    "c4": "3D thermosensitive spheres: D3Q19+D3Q7, 384^3, 20000 spheres D=10, Gr=100",
}
STORAGE_BYTES = {"f32": 4, "f64": 8, "f16": 2, "bf16": 2}


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("pibm_device.h", "pibm.hip"):
        with open(os.path.join(ROOT, "paper_1502_01159_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, storage: str):
    """HBM bytes per launch of the lattice kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_lbm_{workload}_{storage}_traffic.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != source_hash():
        return None
    return float(b.group(1))


def time_gpu(cfg, P, storage, steps, warmup, profile):
    import torch

    from paper_1502_01159_amd import pibm

    sim = pibm.Simulation(cfg, P, storage=storage)
    sim.step(warmup)
    if sim.sync() != pibm.OK:
        raise RuntimeError(f"watchdog during warm-up ({storage})")
    if profile:
        sim.profile(True)
        sim.profile_read()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    sim.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = sim.sync()
    if st != pibm.OK:
        raise RuntimeError(f"watchdog during the timed steps ({storage}): {pibm.strerror(st)}")
    ms = ev0.elapsed_time(ev1)
    prof = sim.profile_read() if profile else None
    out = dict(ms=ms, wall_s=wall, N=sim.N, Q=sim.Q, Qg=sim.Qg, markers=sim.num_markers, prof=prof)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def copy_probe(nbytes=1 << 30, reps=10):
    """A plain device copy of known size (one elementwise kernel: every byte
    read once and written once).  Gives the box's achievable copy bandwidth
    and, under rocprofv3 --pmc, the scale of the FETCH_SIZE / WRITE_SIZE
    counters."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return dict(bytes_per_launch=2 * nbytes, ms=round(ms, 4), GBs=round(2 * nbytes / (ms * 1e-3) / 1e9, 1))


def cpu_baseline(cfg, P, steps):
    from oracle import oracle as O

    t0 = time.perf_counter()
    o = O.Oracle(cfg, P)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.step(steps)
    t = time.perf_counter() - t0
    n = o.N
    del o
    return dict(value=n * steps / t / 1e6, unit="MLUPS", cores=O.num_threads(), kind="oracle",
                sample=f"{steps} full coupled steps of the same workload ({n} nodes, {len(P)} particles), "
                       f"FP64, after {t_init:.1f} s of set-up",
                seconds=round(t, 3))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGE_BYTES))
    ap.add_argument("--variants", default="f16,bf16", help="extra storage formats timed beside the main one")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--empty", action="store_true", help="analysis: the same lattice without particles")
    ap.add_argument("--no-copy-probe", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the lattice would shard as z-slabs with halo exchange; not built).", file=sys.stderr)
        return 2

    from paper_1502_01159_amd import workloads as W

    cfg, P = W.workload(args.workload)
    if args.empty:
        P = P[:0]
    main_run = time_gpu(cfg, P, args.storage, args.steps, args.warmup, profile=True)
    N, Q, Qg = main_run["N"], main_run["Q"], main_run["Qg"]
    ms_step = main_run["ms"] / args.steps
    mlups = N * args.steps / (main_run["ms"] * 1e-3) / 1e6
    bytes_node = 2 * (Q + Qg) * STORAGE_BYTES[args.storage]

    lat_ms, lat_n = main_run["prof"]["lattice"]
    lat_avg_s = lat_ms * 1e-3 / max(lat_n, 1)
    algo_bytes = N * bytes_node                       # one launch updates every node once
    achieved = algo_bytes / lat_avg_s / 1e9
    phases = {k: round(v[0] / max(v[1], 1), 4) for k, v in main_run["prof"].items()}

    variants = {}
    for st in [s for s in args.variants.split(",") if s and s != args.storage]:
        r = time_gpu(cfg, P, st, max(args.steps // 2, 10), args.warmup, profile=True)
        lms, ln = r["prof"]["lattice"]
        n_steps = max(args.steps // 2, 10)
        b = 2 * (Q + Qg) * STORAGE_BYTES[st]
        variants[st] = dict(value=round(N * n_steps / (r["ms"] * 1e-3) / 1e6, 1), unit="MLUPS",
                            ms_per_step=round(r["ms"] / n_steps, 4),
                            lattice_kernel_ms=round(lms / max(ln, 1), 4),
                            lattice_kernel_GBs=round(N * b / (lms * 1e-3 / max(ln, 1)) / 1e9, 1),
                            bytes_per_node=b)

    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "nodes": N, "particles": len(P),
                   "markers": main_run["markers"], "storage": args.storage, "n_sub": cfg["n_sub"]},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_lbm (fused stream + PIBM spreading + forced BGK, f and g)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": read_traffic(args.workload, args.storage),
            "algorithmic_bytes_per_launch": algo_bytes,
            "avg_launch_ms": round(lat_avg_s * 1e3, 4),
        },
        "whole_step_hbm_frac": round(mlups * 1e6 * bytes_node / (HBM_PEAK_GBS * 1e9), 4),
        "phase_ms_per_step": phases,
        "variants": variants,
    }
    if not args.no_copy_probe:
        line["device_copy"] = copy_probe()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, P, args.cpu_steps)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
