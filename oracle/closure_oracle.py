"""FP64 reference of the learned closure's features and targets.

TEST INFRASTRUCTURE ONLY: written from the definitions (block averages of the
raw moments, linear interpolation at the centre, the slip frame, nearest
neighbours by full search) to check the GPU kernels; only tests/ and the
benchmark's CPU leg import it.  It shares no code with the HIP library.

Definitions (one row per particle, D = 2R):
  fluid seen: rho, j, S summed over blocks of b^d nodes (block I covers nodes
    b I .. b I + b - 1 per axis; wrapped on periodic axes, nodes outside a
    wall dropped), u_blk = sum j / sum rho, T_blk = sum S / count, then
    linear interpolation between the 2^d block centres b I + (b - 1)/2
    around the particle centre, renormalised over blocks that hold nodes;
  slip s = U_f - U_p; e1 = s/|s| (|s| = 0: the up axis); 3D: e2 = the up
    axis z (x if |e1_z| > 0.999) minus its e1 part, normalised, e3 = e1 x e2;
    2D: e2 = (-e1_y, e1_x);
  x = [|s| D/nu, g beta (T_p - T_f) D^3 / nu^2, phi, T_p - T_f,
       offsets/D of the 4 (2D: 6) nearest centres in (e1, e2, e3) (2D: e1,
       e2), missing ones at 4], phi = volume (area) of the particles whose
       centres are within 2D (minimum image), self included, over the ball
       (disk) of radius 2D;
  t = [F.e1, F.e2, F.e3 (2D: 0)] / nu^2, H / (pi D alpha) (2D: H/(pi alpha)).
"""
from __future__ import annotations

import math

import numpy as np


def slip_frame(s, dim):
    m = math.sqrt(float(s[0] ** 2 + s[1] ** 2 + s[2] ** 2))
    e1 = np.array(s, dtype=float) / m if m > 1e-300 else np.eye(3)[dim - 1].astype(float)
    if dim == 2:
        return e1, np.array([-e1[1], e1[0], 0.0]), np.array([0.0, 0.0, 1.0])
    up = np.array([0.0, 0.0, 1.0]) if abs(e1[2]) <= 0.999 else np.array([1.0, 0.0, 0.0])
    v = up - up.dot(e1) * e1
    e2 = v / np.linalg.norm(v)
    return e1, e2, np.cross(e1, e2)


def features(rho, j, S, shape, per, P, b, nu, gbeta, dim):
    """rho (N), j (N, 3), S (N) absolute raw moments on a lattice of
    shape (nz, ny, nx); P particle rows (x[3], u[3], ..., R at 12, T at 14 of
    the 16-column particle state).  Returns (x (n, 16), slips (n, 3), T_f)."""
    nz, ny, nx = shape
    nn = (nx, ny, nz)
    rho = rho.reshape(shape)
    jj = j.reshape(shape + (3,))
    SS = S.reshape(shape)
    npart = len(P)
    X = np.zeros((npart, 16))
    slips = np.zeros((npart, 3))
    Tfs = np.zeros(npart)
    NN = 4 if dim == 3 else 6
    for p in range(npart):
        c = P[p, 0:3]
        Up = P[p, 3:6]
        R, Tp = P[p, 12], P[p, 14]
        D = 2 * R
        lo, fr = [0, 0, 0], [0.0, 0.0, 0.0]
        for d in range(dim):
            v = (c[d] - 0.5 * (b - 1)) / b
            lo[d] = math.floor(v)
            fr[d] = v - lo[d]
        acc = np.zeros(4)
        wsum = 0.0
        for k in range(1 << dim):
            kb = [(k >> d) & 1 for d in range(3)]
            w = 1.0
            for d in range(dim):
                w *= fr[d] if kb[d] else 1 - fr[d]
            sr, sj, sS, cnt = 0.0, np.zeros(3), 0.0, 0
            ranges = []
            for d in range(3):
                if d >= dim:
                    ranges.append([0])
                    continue
                idx = []
                for o in range(b):
                    v = (lo[d] + kb[d]) * b + o
                    if per[d]:
                        v %= nn[d]
                    elif v < 0 or v >= nn[d]:
                        continue
                    idx.append(v)
                ranges.append(idx)
            for z in ranges[2]:
                for y in ranges[1]:
                    for x in ranges[0]:
                        sr += rho[z, y, x]
                        sj += jj[z, y, x]
                        sS += SS[z, y, x]
                        cnt += 1
            if cnt:
                acc[:3] += w * sj / sr
                acc[3] += w * sS / cnt
                wsum += w
        Uf = acc[:3] / wsum
        Tf = acc[3] / wsum
        if dim == 2:
            Uf[2] = 0.0
        s = Uf - Up
        if dim == 2:
            s[2] = 0.0
        e1, e2, e3 = slip_frame(s, dim)
        # neighbours
        rphi = 2 * D
        vol = 0.0
        cand = []
        for q in range(npart):
            dx = P[q, 0:3] - c
            for d in range(dim):
                if per[d]:
                    dx[d] -= nn[d] * np.rint(dx[d] / nn[d])
            if dim == 2:
                dx[2] = 0.0
            d2 = float(dx.dot(dx))
            if d2 < rphi * rphi:
                vol += (4 / 3 * math.pi * P[q, 12] ** 3) if dim == 3 else math.pi * P[q, 12] ** 2
            if q != p:
                cand.append((d2, q, dx))
        cand.sort(key=lambda t: (t[0], t[1]))
        x = np.zeros(16)
        x[0] = np.linalg.norm(s) * D / nu
        x[1] = gbeta * (Tp - Tf) * D ** 3 / nu ** 2
        x[2] = vol / ((4 / 3 * math.pi * rphi ** 3) if dim == 3 else math.pi * rphi ** 2)
        x[3] = Tp - Tf
        for q in range(NN):
            o = np.array([4.0, 4.0, 4.0])
            if q < len(cand):
                dx = cand[q][2]
                o = np.array([dx.dot(e1), dx.dot(e2), dx.dot(e3)]) / D
            if dim == 3:
                x[4 + 3 * q:7 + 3 * q] = o
            else:
                x[4 + 2 * q:6 + 2 * q] = o[:2]
        X[p] = x
        slips[p] = s
        Tfs[p] = Tf
    return X, slips, Tfs


def targets(F, H, slips, R, nu, alpha, dim):
    t = np.zeros((len(F), 4))
    for p in range(len(F)):
        e1, e2, e3 = slip_frame(slips[p], dim)
        t[p, 0] = F[p].dot(e1) / nu ** 2
        t[p, 1] = F[p].dot(e2) / nu ** 2
        t[p, 2] = F[p].dot(e3) / nu ** 2 if dim == 3 else 0.0
        t[p, 3] = H[p] / (math.pi * (2 * R[p] if dim == 3 else 1.0) * alpha)
    return t
