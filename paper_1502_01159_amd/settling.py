"""Settling statistics of the 3D sedimentation case across Grashof numbers.

Sec. 3.3 judges the overall sedimentation by the lowest particle height over
time and finds that buoyancy of the fluid heated by hot particles delays the
settling.  Sedimentation is chaotic, so runs that round differently agree
only statistically beyond a short horizon; this module records, every `every`
steps, the lowest particle bottom (z - R), the mean centre height and the
mean vertical particle velocity, for one run or a sweep over Gr.  All the
arithmetic runs in the library's kernels; this module only reads particle
states.
"""
from __future__ import annotations

import numpy as np

from . import workloads as W


def history(pibm, cfg, P, steps, every, storage="f32"):
    """(k, 4) rows: step, lowest bottom z - R, mean centre z, mean u_z."""
    dim = cfg["dim"]
    sim = pibm.Simulation(cfg, P, storage=storage)
    out = []
    for s in range(every, steps + 1, every):
        sim.step(every)
        if sim.sync() != pibm.OK:
            sim.close()
            raise RuntimeError(f"watchdog at step {s}")
        q, _ = sim.particles()
        z = q[:, dim - 1]
        out.append((s, float((z - q[:, 12]).min()), float(z.mean()), float(q[:, 3 + dim - 1].mean())))
    sim.close()
    return np.array(out)


def gr_sweep(pibm, base="c3", grs=(0, 100, 1000), steps=6000, every=250, storage="f32", log=print):
    """Settling histories of workload `base` at each Gr (same placement)."""
    res = {}
    for gr in grs:
        cfg, P = W.workload(f"{base}_gr{gr}")
        h = history(pibm, cfg, P, steps, every, storage)
        res[gr] = h
        for r in h:
            log(f"Gr {gr} step {int(r[0])}: lowest bottom {r[1]:.2f} mean height {r[2]:.2f} mean w {r[3]:+.5f}")
    return res


if __name__ == "__main__":
    import sys

    from . import pibm

    base = sys.argv[1] if len(sys.argv) > 1 else "c3"
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else 6000
    gr_sweep(pibm, base=base, steps=steps)
