"""Seeded synthetic workloads: lattice/physics configurations and particle placements.

This module generates *inputs* only.  It holds none of the method's arithmetic
(no relaxation times, equilibria, forcing or contact laws); both the HIP
library and the CPU oracle receive its plain dicts and arrays and derive
everything else themselves.

The cases stand in for the paper's four studies (Sec. 3): the 2D cavity with a
hot concentric cylinder (Sec. 3.1, Table 1 case Ra = 1e4, Ar = 2.5), 2D and 3D
sedimentation of hot isothermal particles (Secs. 3.2, 3.3) and 3D
thermosensitive particles (Sec. 3.4).  All values are lattice units; gravity
points along -y in 2D and -z in 3D; every non-periodic face is a no-slip wall.

Particle arrays are (n, 13) float64 rows: x[3] u[3] omega[3] R rho_r T flags,
flags = 1 (fixed body) | 2 (thermosensitive).

Random numbers come from splitmix64 (Steele, Lea & Flood, 2014) mapped to
53-bit uniform doubles, so that the placements are reproducible on any host.
"""
from __future__ import annotations

import copy
import math

import numpy as np

FIXED = 1
THERMO = 2

_M64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64: state += golden gamma; output = mix(state)."""

    def __init__(self, seed: int):
        self.state = seed & _M64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniforms(self, n: int) -> np.ndarray:
        return np.array([self.uniform() for _ in range(n)], dtype=np.float64)


def _row(x, R, rho_r, T, flags, u=(0.0, 0.0, 0.0), om=(0.0, 0.0, 0.0)):
    return [x[0], x[1], x[2], u[0], u[1], u[2], om[0], om[1], om[2], R, rho_r, T, float(flags)]


def rsa(seed: int, n: int, lo, hi, min_dist: float, max_trials: int = 2_000_000) -> np.ndarray:
    """Random sequential addition: centres uniform in the box [lo, hi] (per
    axis), accepted when no earlier centre is closer than ``min_dist``."""
    rng = SplitMix64(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    d = lo.size
    pts = np.empty((n, d))
    k = 0
    trials = 0
    md2 = min_dist * min_dist
    while k < n:
        trials += 1
        if trials > max_trials:
            raise RuntimeError(f"RSA could not place {n} particles (placed {k})")
        c = lo + (hi - lo) * np.array([rng.uniform() for _ in range(d)])
        if k:
            dd = pts[:k] - c
            if np.min(np.einsum("ij,ij->i", dd, dd)) < md2:
                continue
        pts[k] = c
        k += 1
    return pts


# --------------------------------------------------------------------------- #
# Base configurations                                                          #
# --------------------------------------------------------------------------- #

def annulus_2d(n: int = 64, Ra: float = 1e4, Ar: float = 2.5, Pr: float = 0.71):
    """Square cavity of side n with a fixed hot cylinder of diameter n/Ar at the
    centre (Sec. 3.1): walls T = 0, cylinder T = 1, fluid initially 0.5,
    Ma = 0.1 (uc = 0.1 c_s)."""
    cfg = dict(
        name=f"annulus2d_{n}", dim=2, nx=n, ny=n, nz=1, periodic=[0, 0, 0],
        T_wall=[0.0] * 6, T_init=0.5, T_ref=0.5,
        Ra=Ra, Pr=Pr, Lc=float(n), uc=0.1 / math.sqrt(3.0), dT_ref=1.0,
        gravity=0.0, kappa_T=1.0, marker_mode=1, marker_spacing=1.0,
        E_star=0.0, poisson=0.33, mu_fric=0.3, n_sub=1, beta_p=0.0, c_r=1.0,
    )
    c = 0.5 * n - 0.5
    P = np.array([_row((c, c, 0.0), 0.5 * n / Ar, 1.0, 1.0, FIXED)])
    return cfg, P


def sediment_2d(nx: int = 512, ny: int = 1024, n_disks: int = 100, D: float = 20.0, seed: int = 2,
                Gr: float = 500.0):
    """2D sedimentation of hot isothermal disks (Sec. 3.2 stand-in): disks
    seeded uniformly without overlap in the upper half."""
    cfg = dict(
        name=f"sediment2d_{nx}x{ny}_{n_disks}", dim=2, nx=nx, ny=ny, nz=1, periodic=[0, 0, 0],
        T_wall=[0.0] * 6, T_init=0.0, T_ref=0.0,
        Ra=0.0, nu=0.04, Pr=0.7, Gr=Gr, Lc=D,
        gravity=0.0125, kappa_T=1.0, marker_mode=1, marker_spacing=1.0,
        E_star=52.6, poisson=0.33, mu_fric=0.3, n_sub=6, beta_p=0.0, c_r=1.0,
    )
    R = 0.5 * D
    lo = [R + 1.0, ny / 2 + R + 1.0]
    hi = [nx - R - 2.0, ny - R - 2.0]
    pts = rsa(seed, n_disks, lo, hi, D + 1.0)
    P = np.array([_row((p[0], p[1], 0.0), R, 1.01, 1.0, 0) for p in pts])
    return cfg, P


def sediment_3d(nx: int = 256, ny: int = 256, nz: int = 512, n_spheres: int = 2000, D: float = 12.0,
                seed: int = 3, Gr: float = 100.0):
    """3D sedimentation of hot isothermal spheres (Sec. 3.3 stand-in): random
    sequential addition in the top third-plus of the box."""
    cfg = dict(
        name=f"sediment3d_{nx}x{ny}x{nz}_{n_spheres}", dim=3, nx=nx, ny=ny, nz=nz, periodic=[0, 0, 0],
        T_wall=[0.0] * 6, T_init=0.0, T_ref=0.0,
        Ra=0.0, nu=0.025, Pr=0.7, Gr=Gr, Lc=D,
        gravity=4.167e-3, kappa_T=1.0, marker_mode=1, marker_spacing=1.0,
        E_star=729.0, poisson=0.33, mu_fric=0.3, n_sub=9, beta_p=0.0, c_r=1.0,
    )
    R = 0.5 * D
    lo = [R + 1.0, R + 1.0, nz * 0.68]
    hi = [nx - R - 2.0, ny - R - 2.0, nz - R - 2.0]
    pts = rsa(seed, n_spheres, lo, hi, D + 1.0)
    P = np.array([_row(p, R, 1.05, 1.0, 0) for p in pts])
    return cfg, P


def thermo_3d(n: int = 384, n_spheres: int = 20000, D: float = 10.0, seed: int = 4, Gr: float = 100.0,
              rho_r: float = 1.25):
    """3D thermosensitive spheres (Sec. 3.4 stand-in): a jittered lattice of
    sites filling the upper part of the box, a seeded subset of them kept,
    initial particle temperature uniform in [0, 1).

    Density ratio 1.25 (the case leaves it open).  At 1.05, as for the heated
    spheres of the sedimentation case, the explicit point exchange amplifies
    the spin of these D = 10 spheres, whose layers start 1 lu apart, by about
    6% a step, and runs diverge within 250 steps; at 1.15 and 1.25 they run
    the case's 5000 steps.  Gravity is scaled so that (rho_r - 1) g, which
    sets the settling speed, stays that of the sedimentation case."""
    cfg = dict(
        name=f"thermo3d_{n}_{n_spheres}", dim=3, nx=n, ny=n, nz=n, periodic=[0, 0, 0],
        T_wall=[0.0] * 6, T_init=0.5, T_ref=0.5,
        Ra=0.0, nu=0.025, Pr=0.7, Gr=Gr, Lc=D,
        gravity=4.167e-3 * 0.05 / (rho_r - 1.0), kappa_T=1.0, marker_mode=1, marker_spacing=1.0,
        E_star=729.0, poisson=0.33, mu_fric=0.3, n_sub=11, beta_p=0.05, c_r=1.0,
    )
    R = 0.5 * D
    lateral = max(1, int(n / (D + 3.714)))           # 28 sites across 384 lu
    pitch = n / lateral
    zpitch = D + 1.0
    top = n - R - 2.0 - 0.5
    layers = int((top - 0.5 * n) / zpitch) + 1 if n_spheres > lateral * lateral else 1
    while lateral * lateral * layers < n_spheres:
        layers += 1
    sites = []
    for m in range(layers):
        z = top - zpitch * m
        for j in range(lateral):
            for i in range(lateral):
                sites.append((-0.5 + pitch * (i + 0.5), -0.5 + pitch * (j + 0.5), z))
    sites = np.array(sites)
    if sites[:, 2].min() - R < 0:
        raise ValueError("lattice of sites does not fit the box")
    rng = SplitMix64(seed)
    # seeded permutation (Fisher-Yates) to choose the kept sites
    idx = list(range(len(sites)))
    for i in range(len(idx) - 1, 0, -1):
        j = int(rng.uniform() * (i + 1))
        idx[i], idx[j] = idx[j], idx[i]
    keep = sorted(idx[:n_spheres])
    P = []
    for s in keep:
        x = sites[s] + (np.array([rng.uniform(), rng.uniform(), rng.uniform()]) - 0.5)
        P.append(_row(x, R, rho_r, rng.uniform(), THERMO))
    return cfg, np.array(P)


def planted_2d(heat: bool = True, n: int = 100, n_particles: int = 5000, d: float = 0.25, gap: float = 0.05,
               seed: int = 21, nu_water: float = 1.0e-6, h_m: float = 1.0e-4, g_si: float = 9.8):
    """A seeded stand-in for the paper's 2D sedimentation of sub-grid
    particles (Sec. 3.2): a 1 cm square cavity on an n x n mesh (h = 0.01 cm)
    with four cold walls, fluid initially at 0.5, and n_particles particles
    of diameter d = h / 4 at seeded random non-overlapping positions (RSA, at
    least d + gap apart and from the walls) in the upper 3/5 of the cavity;
    the paper's own positions come from another study and are not available.
    T_p = 1, density ratio 1.01, Ra = 1e4, Pr = 0.71, L_c = n, u_c = 0.25; one
    point per particle with A_p = d per unit depth; temperature on the flow
    lattice (D2Q9 with the quadratic equilibrium).  `heat=False` switches the
    thermal buoyancy off.  Units and contacts as in planted_3d.

    As printed, the point exchange is unstable here as in the 3D case: one
    step multiplies a point particle's slip by 1 - 8 h / (pi rho_r d) = -9.09
    (Eqs. lbm7, lbm8 with A_p = d and m = rho_r pi d^2 / 4), so the case serves
    for short parity runs."""
    Ra, Pr, uc = 1e4, 0.71, 0.25
    nu_lu = math.sqrt(Pr) * n * uc / math.sqrt(Ra)
    dt = nu_lu * h_m * h_m / nu_water
    cfg = dict(
        name=f"planted2d_{n}_{n_particles}" + ("" if heat else "_noheat"), dim=2, nx=n, ny=n, nz=1,
        periodic=[0, 0, 0], T_wall=[0.0] * 6, T_init=0.5, T_ref=0.5,
        Ra=Ra, Pr=Pr, Lc=float(n), uc=uc, dT_ref=1.0,
        gravity=g_si * dt * dt / h_m, kappa_T=1.0, marker_mode=2, marker_spacing=1.0,
        E_star=40.0, poisson=0.33, mu_fric=0.3, n_sub=20, beta_p=0.0, c_r=1.0, skin=0.15,
        thermal_model=1, seconds_per_step=dt,
    )
    if not heat:
        cfg["gbeta"] = 0.0
    R = 0.5 * d
    m = R + gap
    lo = np.array([-0.5 + m, -0.5 + 0.4 * n + m])
    hi = np.array([n - 0.5 - m, n - 0.5 - m])
    pts = rsa(seed, n_particles, lo, hi, d + gap)
    return cfg, np.array([_row((p[0], p[1], 0.0), R, 1.01, 1.0, 0) for p in pts])


def planted_3d(heat: bool = True, n: int = 15, layers: int = 13, per_axis: int = 25, d: float = 0.5,
               gap: float = 0.1, nu_water: float = 1.0e-6, h_m: float = 1.0e-4, g_si: float = 9.8):
    """The paper's fully specified 3D sedimentation (Sec. 3.3): a cube of n^3
    nodes with six cold walls, fluid initially at 0.5, and per_axis^2 x layers
    sub-grid particles of diameter d = h / 2 planted on a regular lattice with
    gap `gap` between neighbours (0.001 cm at h = 0.01 cm), top-aligned with
    half a gap to the walls, T_p = 1, density ratio 1.01.  Ra = 1e4,
    Pr = 0.71, L_c = n, u_c = 0.25 as for the 2D case; one point per
    particle with A_p = pi d^2 / 4; the literal lattices (D3Q15, temperature
    on D3Q15).  `heat=False` switches the thermal buoyancy off.

    Lattice units from the physical ones (a reading): the time step follows
    from the lattice viscosity and water's nu, dt = nu_lu h^2 / nu_water, so
    g = 9.8 m/s^2 becomes g dt^2 / h.  The contacts are softened to E* = 40
    with 20 sub-steps, so that a collision at 0.01 lu/step spans about a
    dozen sub-steps (the printed 68.95 GPa would need thousands).

    As printed, the point exchange is unstable here: one step multiplies a
    point particle's slip by 1 - 3 h / (rho_r d) = -4.94 (Eqs. lbm7, lbm8,
    lbm13 with A_p = pi d^2 / 4 and m = rho_r pi d^3 / 6), so runs diverge
    within a few hundred steps; the case serves for short parity runs."""
    Ra, Pr, uc = 1e4, 0.71, 0.25
    nu_lu = math.sqrt(Pr) * n * uc / math.sqrt(Ra)
    dt = nu_lu * h_m * h_m / nu_water
    cfg = dict(
        name=f"planted3d_{n}_{per_axis * per_axis * layers}" + ("" if heat else "_noheat"), dim=3, nx=n, ny=n, nz=n,
        periodic=[0, 0, 0], T_wall=[0.0] * 6, T_init=0.5, T_ref=0.5,
        Ra=Ra, Pr=Pr, Lc=float(n), uc=uc, dT_ref=1.0,
        gravity=g_si * dt * dt / h_m, kappa_T=1.0, marker_mode=2, marker_spacing=1.0,
        E_star=40.0, poisson=0.33, mu_fric=0.3, n_sub=20, beta_p=0.0, c_r=1.0, skin=0.15,
        lattice=15, thermal_model=1, seconds_per_step=dt,
    )
    if not heat:
        cfg["gbeta"] = 0.0
    pitch = d + gap
    R = 0.5 * d
    P = []
    for k in range(layers):
        z = n - 0.5 - 0.5 * pitch - pitch * k
        for j in range(per_axis):
            for i in range(per_axis):
                P.append(_row((-0.5 + 0.5 * pitch + pitch * i, -0.5 + 0.5 * pitch + pitch * j, z), R, 1.01, 1.0, 0))
    return cfg, np.array(P)


# --------------------------------------------------------------------------- #
# The named workloads                                                          #
def packed_bed(gap: float = 0.02, seed: int = 15):
    """A dense bed for the DEM's contact path: 107 spheres of D = 6 stacked
    body-centred in five layers (5 x 5 and 4 x 4 alternating) on the floor of
    a walled 34 x 34 x 26 box.  A sphere of a 4 x 4 layer sits on four of the
    layer below and under four of the layer above, `gap` apart, so gravity
    closes every gap within tens of steps: up to 256 oblique pair contacts
    and 25 floor contacts at once, with friction and tangential history.
    Seeded small velocities and spins make the contacts slide.  Hot spheres,
    heat exchange and buoyancy as in the 3D sedimentation case.  Density
    ratio 3: spheres this small and light (rho_r 1.5) are unstable under the
    explicit point exchange (their rotation grows about 1.45-fold per step),
    heavier ones are not."""
    D, R = 6.0, 3.0
    a = 1.1 * D                                    # in-layer pitch: in-layer neighbours never touch
    h = math.sqrt((D + gap) ** 2 - 0.5 * a * a)     # layer spacing: diagonal neighbours `gap` apart
    cfg = dict(
        name="packed_bed_107", dim=3, nx=34, ny=34, nz=26, periodic=[0, 0, 0],
        T_wall=[0.0] * 6, T_init=0.0, T_ref=0.0,
        Ra=0.0, nu=0.025, Pr=0.7, Gr=100.0, Lc=D,
        gravity=4.167e-3, kappa_T=1.0, marker_mode=1, marker_spacing=1.0,
        E_star=729.0, poisson=0.33, mu_fric=0.3, n_sub=9, beta_p=0.0, c_r=1.0,
    )
    rng = SplitMix64(seed)
    rows = []
    for k in range(5):
        z = R - 0.5 + gap + k * h
        if k % 2 == 0:
            sites = [(0.5 * a + i * a, 0.5 * a + j * a) for j in range(5) for i in range(5)]
        else:
            sites = [(a + i * a, a + j * a) for j in range(4) for i in range(4)]
        for x, y in sites:
            u = [0.004 * (2 * rng.uniform() - 1) for _ in range(3)]
            om = [0.002 * (2 * rng.uniform() - 1) for _ in range(3)]
            rows.append(_row((x, y, z), R, 3.0, 1.0, 0, u=u, om=om))
    return cfg, np.array(rows)


# --------------------------------------------------------------------------- #

def workload(name: str):
    """Named workloads.  Full sizes:
    c1 annulus 64^2; c2 2D sedimentation 512x1024, 100 disks; c3 3D
    sedimentation 256x256x512, 2000 spheres; c4 thermosensitive 384^3, 20000
    spheres (c3_mid and c4_mid: the same with a box 4 times smaller per
    axis); x2 / x2_noheat a seeded stand-in for the paper's 2D case of 5000
    sub-grid particles on 100^2; x3 / x3_noheat the paper's planted 15^3 case with 8125 point
    particles, with and without thermal buoyancy; packed_bed 107 spheres in
    contact on a floor.  Small variants (suffix _small) keep the structure for parity
    runs that the oracle finishes in seconds."""
    if name == "c1":
        return annulus_2d(64)
    if name == "c2":
        return sediment_2d()
    if name == "c2_small":
        return sediment_2d(nx=96, ny=160, n_disks=6, D=16.0, seed=12)
    if name.startswith("c3"):
        gr = 100.0
        if "_gr" in name:
            gr = float(name.split("_gr")[1])
        if name.startswith("c3_small"):
            return sediment_3d(nx=48, ny=40, nz=64, n_spheres=6, D=10.0, seed=13, Gr=gr)
        if name.startswith("c3_mid"):
            # the 256 x 256 x 512 case with a box 4 times smaller per axis and
            # 32 spheres of the same D = 12 (the same solid fraction of about
            # 0.17 in the seeded top third)
            return sediment_3d(nx=64, ny=64, nz=128, n_spheres=32, D=12.0, seed=5, Gr=gr)
        return sediment_3d(Gr=gr)
    if name == "c4":
        return thermo_3d()
    if name == "c4_small":
        return thermo_3d(n=48, n_spheres=9, D=10.0, seed=14)
    if name == "c4_mid":
        # the 384^3 case with a box 4 times smaller per axis: 6 layers of
        # 7 x 7 sites over the upper three quarters of the height, 288 of the
        # 294 kept (the full case keeps 20000 of 26 x 28 x 28)
        return thermo_3d(n=96, n_spheres=288, D=10.0, seed=16)
    if name == "x2":
        return planted_2d(heat=True)
    if name == "x2_noheat":
        return planted_2d(heat=False)
    if name == "x3":
        return planted_3d(heat=True)
    if name == "x3_noheat":
        return planted_3d(heat=False)
    if name == "packed_bed":
        return packed_bed()
    raise KeyError(name)


def with_overrides(cfg: dict, **kw) -> dict:
    out = copy.deepcopy(cfg)
    out.update(kw)
    return out


def perturbed_populations(seed: int, Q: int, N: int, weights, base: float, amp: float) -> np.ndarray:
    """Random populations w_a (base + amp * U(-1, 1)) for single-step tests
    that start from a non-equilibrium state."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64).reshape(Q, 1)
    return w * (base + amp * (2.0 * rng.random((Q, N)) - 1.0))
