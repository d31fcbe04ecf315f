"""Line footprint of the Lagrangian-point gather (analysis, host only).

The marker kernel pulls the streamed populations at the stencil nodes of
every Lagrangian point: the cell corners floor(X_l) .. floor(X_l) + 1 per axis
for the multilinear interpolation of Eq. (lbm6) (i_max = 2), indices clamped
at walls.  Pulling node x reads population q at x - e_q from q's array, or at
a wall this node's opposite population.  HBM moves whole 128-byte lines, so
the floor of the gather's traffic is the number of distinct lines those reads
touch over all particles, each read once.  This module counts them on the
host from the particle state, with the same sphere templates as the library
(round(pi D^2 / s^2) points on a Fibonacci sphere, spacing s = 1), and
compares them with the bytes the populations themselves hold.
"""
from __future__ import annotations

import math

import numpy as np

from . import workloads as W

# D3Q19 and D3Q7 velocity sets: the rest population, then opposite pairs
_E19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 1, 0), (-1, -1, 0),
        (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1),
        (0, 1, -1), (0, -1, 1)]
_E7 = _E19[:7]


def sphere_points(R, s=1.0):
    D = 2.0 * R
    n = max(1, int(round(math.pi * D * D / (s * s))))
    k = np.arange(n)
    z = 1.0 - (2.0 * k + 1.0) / n
    rr = np.sqrt(1.0 - z * z)
    ph = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([R * rr * np.cos(ph), R * rr * np.sin(ph), R * z], 1)


def shell_nodes(cfg, P):
    """Linear indices of the distinct stencil nodes of all points (3D)."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    parts = []
    for row in P:
        b = np.floor(row[:3] + sphere_points(row[9])).astype(np.int64)
        for o in np.ndindex(2, 2, 2):
            c = b + np.array(o)
            c[:, 0] = np.clip(c[:, 0], 0, nx - 1)
            c[:, 1] = np.clip(c[:, 1], 0, ny - 1)
            c[:, 2] = np.clip(c[:, 2], 0, nz - 1)
            parts.append((c[:, 2] * ny + c[:, 1]) * nx + c[:, 0])
    return np.unique(np.concatenate(parts))


def count(cfg, P, value_bytes=4, line_bytes=128):
    """(shell nodes, distinct lines the pull touches, population bytes of the
    shell, line bytes).  Arrays start on line boundaries (their stride is a
    whole number of lines), so a line is (array, node // nodes per line)."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    per_line = line_bytes // value_bytes
    nodes = shell_nodes(cfg, P)
    x, y, z = nodes % nx, (nodes // nx) % ny, nodes // (nx * ny)
    keys = []
    for first, E in ((0, _E19), (len(_E19), _E7)):
        for q, e in enumerate(E):
            sx, sy, sz = x - e[0], y - e[1], z - e[2]
            inside = (sx >= 0) & (sx < nx) & (sy >= 0) & (sy < ny) & (sz >= 0) & (sz < nz)
            opp = q if q == 0 else (q + 1 if q % 2 else q - 1)
            src = np.where(inside, (sz * ny + sy) * nx + sx, nodes)
            arr = np.where(inside, first + q, first + opp)
            keys.append(arr.astype(np.int64) * (1 << 40) + src // per_line)
    lines = len(np.unique(np.concatenate(keys)))
    return len(nodes), lines, len(nodes) * 26 * value_bytes, lines * line_bytes


if __name__ == "__main__":
    import sys

    for name in sys.argv[1:] or ["c3", "c4"]:
        cfg, P = W.workload(name)
        for vb in (4, 2):
            n, lines, pb, lb = count(cfg, P, vb)
            print(f"{name} ({8 * vb}-bit storage): {len(P)} particles, {n} shell nodes, populations {pb / 1e6:.1f} MB, "
                  f"{lines} distinct 128-byte lines = {lb / 1e6:.1f} MB ({lb / pb:.1f}x)")
