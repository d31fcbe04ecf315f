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
    "c4": "3D thermosensitive spheres: D3Q19+D3Q7, 384^3, 20000 spheres D=10, density ratio 1.25, Gr=100",
}
STORAGE_BYTES = {"f32": 4, "f64": 8, "f16": 2, "bf16": 2}
# storage type of the populations and the type the collision computes in
DTYPE_TEXT = {"f32": "f32 storage, f64 collision", "f64": "f64", "f16": "f16 storage, f32 collision",
              "bf16": "bf16 storage, f32 collision"}


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("pibm_device.h", "pibm.hip"):
        with open(os.path.join(ROOT, "paper_1502_01159_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def two_streams(nodes: int, particles: int) -> int:
    """Streams the library's step uses with pibm_params.streams = 0: two from
    2^22 nodes when there are particles, else one."""
    return 2 if particles > 0 and nodes >= (1 << 22) else 1


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


def time_gpu(cfg, P, storage, steps, warmup, phase_steps=0):
    """Times `steps` steps with events around the lattice kernel only (each
    timed phase adds an event pair to the stream); then, untimed, reads every
    phase's time over `phase_steps` further steps."""
    import torch

    from paper_1502_01159_amd import pibm

    sim = pibm.Simulation(cfg, P, storage=storage)
    sim.step(warmup)
    if sim.sync() != pibm.OK:
        raise RuntimeError(f"watchdog during warm-up ({storage})")
    sim.profile(True, phases=["lattice"])
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
    prof = sim.profile_read()
    all_prof = None
    if phase_steps:
        sim.profile(True)
        sim.step(phase_steps)
        all_prof = sim.profile_read()
        sim.profile(False)
        if sim.sync() != pibm.OK:
            raise RuntimeError(f"watchdog during the phase run ({storage})")
    out = dict(ms=ms, wall_s=wall, N=sim.N, Q=sim.Q, Qg=sim.Qg, markers=sim.num_markers, prof=prof,
               all_prof=all_prof)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def copy_probe(nbytes=1 << 30, reps=10):
    """A plain device copy of known size (one elementwise kernel: every byte
    read once and written once).  Gives the device's achievable copy bandwidth
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


MLP_FLOP_PER_SAMPLE = 2 * (16 * 128 + 128 * 128 + 128 * 128 + 128 * 4)   # forward multiply-adds x 2
BF16_PEAK_TFLOPS = 2500.0


def mlp_variant(steps):
    """The learned part: inference on 10^6 feature rows and one Adam step on a
    batch of 4096 through the matrix-core kernels, and a coarse one-point step
    with the network as the closure (zero weights, so it applies the mean
    drag and Nusselt factors of its normalisation; the kernels do the same
    work whatever the weights)."""
    import numpy as np
    import torch

    from paper_1502_01159_amd import closure as CL, pibm

    out = {}
    n = 1 << 20
    g = torch.Generator(device="cuda").manual_seed(1)
    x = torch.randn((n, 16), device="cuda", generator=g).to(torch.bfloat16)
    y = torch.empty((n, 4), device="cuda", dtype=torch.float32)
    mlp = pibm.Mlp(seed=3, max_batch=4096)
    mlp.forward(x, y)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    ev0.record()
    for _ in range(reps):
        mlp.forward(x, y)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    tf = MLP_FLOP_PER_SAMPLE * n / (ms * 1e-3) / 1e12
    out["inference"] = dict(samples=n, ms=round(ms, 4), samples_per_s=round(n / (ms * 1e-3), 0),
                            TFLOPs=round(tf, 1), frac_bf16_peak=round(tf / BF16_PEAK_TFLOPS, 4))
    tb = torch.randn((4096, 4), device="cuda", generator=g)
    xb = x[:4096].contiguous()
    mlp.train_step(xb, tb, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mlp.train_step(xb, tb, 1e-4)
    torch.cuda.synchronize()
    ms_t = (time.perf_counter() - t0) * 1e3 / reps
    out["train_step"] = dict(batch=4096, ms=round(ms_t, 4),
                             TFLOPs=round(3 * MLP_FLOP_PER_SAMPLE * 4096 / (ms_t * 1e-3) / 1e12, 2))
    # coarse one-point run with the network as the closure
    cfg, P = CL.fixed_array(L=256, n=4000, D=8.0, seed=41)
    cc, Pc = CL.coarsen(cfg, P)
    mlp.set_params(np.zeros(pibm.MLP_NPARAM, dtype=np.float32))
    norm = np.concatenate([np.zeros(16), np.ones(16), [3.5, 0.0, 0.0, 4.2], np.ones(4)]).astype(np.float32)
    sim = pibm.Simulation(cc, Pc, storage="f32")
    sim.set_closure(mlp, norm)
    sim.step(5)
    if sim.sync() != pibm.OK:
        raise RuntimeError("coarse closure run failed in warm-up")
    torch.cuda.synchronize()
    ev0.record()
    sim.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    ms_c = ev0.elapsed_time(ev1) / steps
    sim.profile(True)                     # phase times from further, untimed steps
    sim.step(20)
    prof = {k: round(v[0] / max(v[1], 1), 4) for k, v in sim.profile_read().items()}
    if sim.sync() != pibm.OK:
        raise RuntimeError("coarse closure run failed")
    Nc, Nf = sim.N, cfg["nx"] * cfg["ny"] * cfg["nz"]
    out["coarse_step"] = dict(workload=f"fixed hot spheres, {cc['nx']}^3 coarse lattice (256^3 resolved / 4), "
                                       f"{len(P)} one-point particles, network closure",
                              ms_per_step=round(ms_c, 4), coarse_MLUPS=round(Nc / (ms_c * 1e-3) / 1e6, 1),
                              resolved_equivalent_MLUPS=round(Nf * 16 / (ms_c * 1e-3) / 1e6, 1),
                              phase_ms_per_step=prof)
    sim.set_closure(None)
    sim.close()
    mlp.close()
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, P, steps):
    """The FP64 oracle on the host cores: `steps` full coupled steps with all
    threads, then one step with one thread (each after the same set-up)."""
    from oracle import oracle as O

    t0 = time.perf_counter()
    o = O.Oracle(cfg, P)
    t_init = time.perf_counter() - t0
    threads = O.num_threads()
    t0 = time.perf_counter()
    o.step(steps)
    t = time.perf_counter() - t0
    n = o.N
    O.set_threads(1)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    O.set_threads(threads)
    del o
    return dict(value=n * steps / t / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{steps} full coupled steps of the same workload ({n} nodes, {len(P)} particles), "
                       f"FP64, after {t_init:.1f} s of set-up",
                seconds=round(t, 3),
                single_thread=dict(value=round(n / t1 / 1e6, 3), unit="MLUPS", cores=1, seconds=round(t1, 3),
                                   sample="1 further full coupled step of the same run, one thread"),
                cpu_model=cpu_model(), nproc=os.cpu_count())


def storage_errors(cfg, P, storages, steps):
    """Field errors of each storage format against the FP64 path on the same
    workload after `steps` steps (the FP64 path is held to 1e-9 of the FP64
    oracle by the parity tests): max |a - b| / max |b| for rho, for u (all
    components) and for T."""
    import numpy as np
    import torch

    from paper_1502_01159_amd import pibm

    def run(st):
        sim = pibm.Simulation(cfg, P, storage=st)
        sim.step(steps)
        if sim.sync() != pibm.OK:
            raise RuntimeError(f"watchdog in the {st} error run")
        out = sim.fields()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        return out

    ref = run("f64")
    errs = {}
    for st in storages:
        got = run(st)
        errs[st] = {k: float(f"{np.abs(a - b).max() / max(np.abs(b).max(), 1e-30):.3e}")
                    for k, a, b in zip(("rho", "u", "T"), got, ref)}
        errs[st]["meets_1e-3"] = bool(errs[st]["u"] <= 1e-3 and errs[st]["T"] <= 1e-3)
    return errs


def graph_time(cfg, P, storage, steps, warmup):
    """The step replayed from a HIP graph (timing only): two steps are captured
    on a stream of their own (an even count returns every double buffer to
    its place) and replayed.  The replays reuse the captured step counter, so
    the stochastic-rounding stream repeats every two steps: the timing is
    meaningful, the trajectory is not the eager one."""
    import torch

    from paper_1502_01159_amd import pibm

    s = torch.cuda.Stream()
    sim = pibm.Simulation(cfg, P, storage=storage, stream=s)
    sim.step(warmup)
    if sim.sync() != pibm.OK:
        raise RuntimeError("watchdog before capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        sim.step(2)
    torch.cuda.synchronize()
    reps = max(steps // 2, 1)
    with torch.cuda.stream(s):
        g.replay()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(reps):
            g.replay()
        ev1.record(s)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / (2 * reps)
    ok = sim.sync() == pibm.OK
    sim.close()
    return dict(ms_per_step=round(ms, 4), steps=2 * reps, watchdog_ok=ok)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGE_BYTES))
    ap.add_argument("--variants", default="f16,bf16,q15,literal,c4,mlp",
                    help="extra storage formats timed beside the main one, 'q15' for the D3Q15 flow lattice "
                         "(FP32, 3D workloads), 'literal' for D3Q15 with temperature on the flow lattice "
                         "(quadratic equilibrium, FP32), 'c4' for the 384^3 thermosensitive workload (FP32) "
                         "and 'mlp' for the learned part")
    ap.add_argument("--error-steps", type=int, default=300,
                    help="steps after which each storage format's fields are compared with the FP64 path (0: off)")
    ap.add_argument("--graph", action="store_true", help="also time the step replayed from a HIP graph")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--empty", action="store_true", help="analysis: the same lattice without particles")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--streams", type=int, default=0, choices=(0, 1, 2),
                    help="pibm_params.streams: 0 automatic, 1 one stream, 2 two streams")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the lattice would shard as z-slabs with halo exchange; not built).", file=sys.stderr)
        return 2

    from paper_1502_01159_amd import workloads as W

    cfg, P = W.workload(args.workload)
    if args.streams:
        cfg = W.with_overrides(cfg, streams=args.streams)
    if args.empty:
        P = P[:0]
    main_run = time_gpu(cfg, P, args.storage, args.steps, args.warmup, phase_steps=20)
    N, Q, Qg = main_run["N"], main_run["Q"], main_run["Qg"]
    ms_step = main_run["ms"] / args.steps
    mlups = N * args.steps / (main_run["ms"] * 1e-3) / 1e6
    bytes_node = 2 * (Q + Qg) * STORAGE_BYTES[args.storage]

    lat_ms, lat_n = main_run["prof"]["lattice"]
    lat_avg_s = lat_ms * 1e-3 / max(lat_n, 1)
    algo_bytes = N * bytes_node                       # one launch updates every node once
    achieved = algo_bytes / lat_avg_s / 1e9
    phases = {k: round(v[0] / max(v[1], 1), 4) for k, v in main_run["all_prof"].items()}

    variants = {}
    for st in [s for s in args.variants.split(",") if s and s != args.storage and s not in ("mlp", "c4")]:
        if st in ("q15", "literal") and cfg["dim"] != 3:
            continue
        if st == "q15":
            vcfg, vst = W.with_overrides(cfg, lattice=15), "f32"
        elif st == "literal":
            vcfg, vst = W.with_overrides(cfg, lattice=15, thermal_model=1), "f32"
        else:
            vcfg, vst = cfg, st
        r = time_gpu(vcfg, P, vst, max(args.steps // 2, 10), args.warmup)
        lms, ln = r["prof"]["lattice"]
        n_steps = max(args.steps // 2, 10)
        b = 2 * (r["Q"] + r["Qg"]) * STORAGE_BYTES[vst]
        variants[st] = dict(value=round(N * n_steps / (r["ms"] * 1e-3) / 1e6, 1), unit="MLUPS",
                            ms_per_step=round(r["ms"] / n_steps, 4),
                            lattice_kernel_ms=round(lms / max(ln, 1), 4),
                            lattice_kernel_GBs=round(N * b / (lms * 1e-3 / max(ln, 1)) / 1e9, 1),
                            bytes_per_node=b)

    if "c4" in args.variants.split(",") and args.workload == "c3" and not args.empty:
        c4cfg, c4P = W.workload("c4")
        n4 = max(args.steps // 2, 10)
        r = time_gpu(c4cfg, c4P, "f32", n4, args.warmup)
        lms, ln = r["prof"]["lattice"]
        b = 2 * (r["Q"] + r["Qg"]) * STORAGE_BYTES["f32"]
        gbs = r["N"] * b / (lms * 1e-3 / max(ln, 1)) / 1e9
        variants["c4"] = dict(workload=WORKLOAD_TEXT["c4"], storage="f32",
                              value=round(r["N"] * n4 / (r["ms"] * 1e-3) / 1e6, 1), unit="MLUPS",
                              ms_per_step=round(r["ms"] / n4, 4), lattice_kernel_ms=round(lms / max(ln, 1), 4),
                              lattice_kernel_GBs=round(gbs, 1), lattice_kernel_frac=round(gbs / HBM_PEAK_GBS, 4),
                              bytes_per_node=b)
    errs = None
    err_st = [st for st in ("f32", "f16", "bf16") if st in args.variants.split(",") or st == args.storage]
    if args.error_steps > 0 and err_st and not args.empty:
        errs = storage_errors(cfg, P, err_st, args.error_steps)
    graph = None
    if args.graph or (args.workload == "c2" and not args.empty):
        graph = graph_time(cfg, P, args.storage, args.steps, args.warmup)
        graph["eager_ms_per_step"] = round(ms_step, 4)

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
        "dtype": DTYPE_TEXT[args.storage],
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "nodes": N, "particles": len(P),
                   "markers": main_run["markers"], "storage": args.storage, "n_sub": cfg["n_sub"],
                   "streams": args.streams or two_streams(N, len(P))},
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
        "phase_note": ("phase times from 20 further steps with events around every phase (the timed steps carry "
                       "events around the lattice kernel only); " +
                       ("two streams: binning runs beside the markers and the DEM beside the lattice, so the phase "
                        "spans overlap and sum to more than ms_per_step"
                        if (args.streams or two_streams(N, len(P))) == 2 else
                        "one stream: the phases run one after another")),
        "variants": variants,
    }
    if errs is not None:
        line["storage_error_vs_f64"] = dict(steps=args.error_steps, bar=1e-3, fields=errs,
                                            note="fields after the same number of steps against the FP64 path "
                                                 "on the same workload; the bar applies to u and T")
    if graph is not None:
        line["graph_replay"] = graph
    if "mlp" in [v for v in args.variants.split(",") if v]:
        line["mlp"] = mlp_variant(max(args.steps // 2, 10))
    if not args.no_copy_probe:
        line["device_copy"] = copy_probe()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, P, args.cpu_steps)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
