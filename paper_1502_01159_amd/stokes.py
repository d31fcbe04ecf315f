"""Stokes drag on a fixed sphere in a periodic box (a simple cubic array),
the fluid driven by a uniform force: at Re << 1 the drag and the mean fluid
velocity U obey F = 6 pi mu a U K(phi), with Hasimoto's array factor K
(Hasimoto 1959, in the form K = 1 / (1 - 1.7601 phi^(1/3) + phi - 1.5593
phi^2)).  The hydrodynamic radius a of the diffuse PIBM body is reported
against the point radius R.

    python -m paper_1502_01159_amd.stokes [--L 96] [--R 6] [--interp-order 2|4] [--marker-mode 0|1]

Every number comes from the library's kernels; this module sets up the run
and reads the drag and the mean velocity.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import workloads as W


def hasimoto_K(phi: float) -> float:
    return 1.0 / (1.0 - 1.7601 * phi ** (1.0 / 3.0) + phi - 1.5593 * phi ** 2)


def run(pibm, L=96, R=6.0, tau=1.0, gbeta=1e-8, interp_order=2, marker_mode=1, steps=(4000, 1000),
        storage="f64"):
    """Returns dict(a, a_over_R, Re, drift): the hydrodynamic radius after
    steps[0] steps and its relative change over steps[1] more."""
    nu = (tau - 0.5) / 3.0
    cfg = dict(dim=3, nx=L, ny=L, nz=L, periodic=[1, 1, 1], T_wall=[0.0] * 6, T_init=1.0, T_ref=0.0, Ra=0.0,
               nu=nu, Pr=0.7, Gr=0.0, Lc=10.0, gbeta=gbeta, gravity=0.0, kappa_T=1.0, marker_mode=marker_mode,
               marker_spacing=1.0, E_star=0.0, poisson=0.33, mu_fric=0.3, n_sub=1, beta_p=0.0, c_r=1.0,
               interp_order=interp_order)
    c = (L - 1) / 2.0
    P = np.array([W._row((c, c, c), R, 1.0, 1.0, W.FIXED)])
    sim = pibm.Simulation(cfg, P, storage=storage)
    phi = 4.0 / 3.0 * math.pi * R ** 3 / L ** 3
    K = hasimoto_K(phi)
    F = gbeta * L ** 3                               # total driving force = drag at steady state
    u0 = F / (6.0 * math.pi * nu * (R + 0.5) * K)   # start the fluid near its steady mean velocity
    ez = np.array([0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1], dtype=float)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    f0, g0 = sim.populations()
    f0[:] = (w * (1.0 + 3.0 * ez * u0 + 4.5 * (ez * u0) ** 2 - 1.5 * u0 ** 2))[:, None]
    sim.set_populations(f0, g0)

    def radius():
        rho, u, T = sim.fields()
        U = float(u[..., 2].mean())
        _, fth = sim.particles()
        return fth[0, 2] / (6.0 * math.pi * nu * K * U), U

    sim.step(steps[0])
    a1, _ = radius()
    sim.step(steps[1])
    a2, U = radius()
    sim.close()
    return dict(L=L, R=R, phi=phi, K=round(K, 4), interp_order=interp_order, marker_mode=marker_mode,
                a=round(a2, 4), a_over_R=round(a2 / R, 4), Re=U * 2 * R / nu, drift=abs(a2 - a1) / a2)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--L", type=int, default=96)
    ap.add_argument("--R", type=float, default=6.0)
    ap.add_argument("--interp-order", type=int, default=2)
    ap.add_argument("--marker-mode", type=int, default=1)
    args = ap.parse_args(argv)
    from . import pibm

    print(json.dumps(run(pibm, args.L, args.R, interp_order=args.interp_order, marker_mode=args.marker_mode)),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
