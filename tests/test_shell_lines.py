"""The marker gather's line floor (host analysis, CPU only).

`shell_lines.count` counts, with numpy, the distinct 128-byte lines that
pulling the populations at every stencil node of every Lagrangian point
touches.  Here the same count is made with plain Python loops over points,
corners and directions on the small walled 3D case, and the velocity sets
are checked against their definitions (Sec. 2.1: D3Q19 and D3Q7 with
opposite directions in adjacent slots).
"""
import math

import numpy as np

from paper_1502_01159_amd import shell_lines as S, workloads as W


def test_velocity_sets():
    e19 = [tuple(e) for e in S._E19]
    assert len(set(e19)) == 19 and e19[0] == (0, 0, 0)
    assert all(sum(c * c for c in e) in (1, 2) for e in e19[1:])
    for q in range(1, 19, 2):
        assert tuple(-c for c in e19[q]) == e19[q + 1]
    assert [tuple(e) for e in S._E7] == e19[:7]


def test_sphere_points_on_the_sphere():
    R = 6.0
    pts = S.sphere_points(R)
    assert len(pts) == round(math.pi * (2 * R) ** 2)
    assert np.allclose(np.linalg.norm(pts, axis=1), R)


def _brute_force(cfg, P, value_bytes, line_bytes=128):
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    dims = (nx, ny, nz)
    nodes = set()
    for row in P:
        for p in S.sphere_points(row[9]):
            base = [math.floor(row[a] + p[a]) for a in range(3)]
            for o in ((i, j, k) for i in (0, 1) for j in (0, 1) for k in (0, 1)):
                nodes.add(tuple(min(max(base[a] + o[a], 0), dims[a] - 1) for a in range(3)))
    per_line = line_bytes // value_bytes
    lines = set()
    arrays = [(q, e) for q, e in enumerate(S._E19)] + [(19 + q, e) for q, e in enumerate(S._E7)]
    for (x, y, z) in nodes:
        for arr, e in arrays:
            src = (x - e[0], y - e[1], z - e[2])
            if all(0 <= src[a] < dims[a] for a in range(3)):
                lin = (src[2] * ny + src[1]) * nx + src[0]
                lines.add((arr, lin // per_line))
            else:
                # a wall: the node's own value of the opposite direction
                q = arr if arr < 19 else arr - 19
                opp = q if q == 0 else (q + 1 if q % 2 else q - 1)
                lin = (z * ny + y) * nx + x
                lines.add((opp + (0 if arr < 19 else 19), lin // per_line))
    return len(nodes), len(lines)


def test_count_matches_loops_on_walled_case():
    cfg, P = W.workload("c3_small")
    for vb in (4, 2):
        n, lines, pop_bytes, line_bytes = S.count(cfg, P, vb)
        bn, blines = _brute_force(cfg, P, vb)
        assert (n, lines) == (bn, blines)
        assert pop_bytes == n * 26 * vb and line_bytes == lines * 128
        # every node's 26 values fill at least their share of whole lines
        assert line_bytes >= pop_bytes
