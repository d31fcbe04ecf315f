"""FP64 reference of the learned closure's features and targets.

TEST INFRASTRUCTURE ONLY: written from the definitions (block averages of the
raw moments, linear interpolation at the centre, the slip frame, nearest
neighbours by full search) to check the GPU kernels; only tests/ and the
benchmark's CPU leg import it.  It shares no code with the HIP library.

Definitions (one row per particle, D = 2R):
  fluid seen: rho, j, S summed over the lattice nodes x with
    0.75 D <= |x - X_p| <= 1.5 D (coordinates unwrapped, then wrapped on
    periodic axes; nodes beyond a wall dropped), U_f = sum j / sum rho,
    T_f = sum S / count;
  slip s = U_f - U_p; e1 = s/|s| (|s| = 0: the up axis); 3D: e2 = the up
    axis z (x if |e1_z| > 0.999) minus its e1 part, normalised, e3 = e1 x e2;
    2D: e2 = (-e1_y, e1_x);
  x = [|s| D/nu, g beta (T_p - T_f) D^3 / nu^2, phi, T_p - T_f,
       offsets/D of the 4 (2D: 6) nearest centres in (e1, e2, e3) (2D: e1,
       e2), missing ones at 4], phi = volume (area) of the particles whose
       centres are within 2D (minimum image), self included, over the ball
       (disk) of radius 2D;
  t = [F.e1, F.e2, F.e3 (2D: 0)] / (3 pi nu D |s|) and the Nusselt number
      H / (pi D alpha (T_p - T_f)) (2D: H / (pi alpha (T_p - T_f))), 0 where
      |s| or T_p - T_f is 0.
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


def features(rho, j, S, shape, per, P, nu, gbeta, dim):
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
        r_in, r_out = 0.75 * D, 1.5 * D
        axes = []
        for d in range(3):
            if d >= dim:
                axes.append([(0, 0.0)])
                continue
            vals = []
            for v0 in range(math.ceil(c[d] - r_out), math.floor(c[d] + r_out) + 1):
                v = v0 % nn[d] if per[d] else v0
                if not per[d] and (v < 0 or v >= nn[d]):
                    continue
                vals.append((v, (v0 - c[d]) ** 2))
            axes.append(vals)
        sr, sj, sS, cnt = 0.0, np.zeros(3), 0.0, 0
        for z, dz in axes[2]:
            for y, dy in axes[1]:
                for x, dx in axes[0]:
                    r2 = dx + dy + dz
                    if r2 < r_in * r_in or r2 > r_out * r_out:
                        continue
                    sr += rho[z, y, x]
                    sj += jj[z, y, x]
                    sS += SS[z, y, x]
                    cnt += 1
        Uf = sj / sr
        Tf = sS / cnt
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


def targets(F, H, slips, R, dT, nu, alpha, dim):
    t = np.zeros((len(F), 4))
    for p in range(len(F)):
        e1, e2, e3 = slip_frame(slips[p], dim)
        D = 2 * R[p]
        fs = 3 * math.pi * nu * D * np.linalg.norm(slips[p])
        hs = math.pi * (D if dim == 3 else 1.0) * alpha * dT[p]
        f = 1.0 / fs if fs > 1e-300 else 0.0
        h = 1.0 / hs if abs(hs) > 1e-300 else 0.0
        t[p, 0] = F[p].dot(e1) * f
        t[p, 1] = F[p].dot(e2) * f
        t[p, 2] = F[p].dot(e3) * f if dim == 3 else 0.0
        t[p, 3] = H[p] * h
    return t
