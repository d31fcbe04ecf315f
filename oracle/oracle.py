"""ctypes front end of the FP64 CPU oracle (``oracle/pibm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the product package.  The oracle
shares no code with the HIP library.  Configurations arrive as the plain dicts
of the workload generator; the relaxation times and the Boussinesq coefficient
are derived here, independently of the HIP library's own derivation:

* Ra-based (Sec. 2.1, Eqs. lbm2.6 and lbm2.7): nu = sqrt(Pr) Lc uc / sqrt(Ra),
  alpha = Lc uc / sqrt(Pr Ra), u_c^2 = g beta Lc dT  =>  g beta = uc^2/(Lc dT);
* Grashof-based (Gr on the particle diameter Lc): alpha = nu / Pr,
  g beta = Gr nu^2 / Lc^3;
* tau_f = nu / (1/3) + 1/2; tau_g = alpha / c_sg^2 + 1/2 with c_sg^2 = 1/3
  (D2Q5) or 1/4 (D3Q7).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpibm_oracle.so")
SRC_PATH = os.path.join(_HERE, "pibm_oracle.c")


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("periodic", ctypes.c_int * 3),
        ("T_wall", ctypes.c_double * 6),
        ("T_init", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double),
        ("gbeta", ctypes.c_double), ("gravity", ctypes.c_double), ("kappa_T", ctypes.c_double),
        ("E_star", ctypes.c_double), ("poisson", ctypes.c_double), ("mu_fric", ctypes.c_double),
        ("n_sub", ctypes.c_int),
        ("beta_p", ctypes.c_double), ("c_r", ctypes.c_double),
        ("marker_mode", ctypes.c_int), ("marker_spacing", ctypes.c_double),
        ("interp_order", ctypes.c_int), ("lattice", ctypes.c_int), ("thermal_model", ctypes.c_int),
    ]


def compile_library(src: str, out: str) -> str:
    """gcc the oracle source ``src`` into the shared library ``out`` (portable
    x86-64 flags, IEEE arithmetic: no fast-math, no FMA contraction)."""
    import subprocess

    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                           "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle next to its source if it is missing or stale."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        compile_library(SRC_PATH, LIB_PATH)
    return LIB_PATH


_lib = None


def load(path: str):
    """Open an oracle library at ``path`` and declare its C signatures."""
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    L.orc_create.restype = vp
    L.orc_create.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_int, dp]
    L.orc_destroy.argtypes = [vp]
    L.orc_step.argtypes = [vp, ctypes.c_int]
    L.orc_dem_only.argtypes = [vp, ctypes.c_int]
    L.orc_clear_reactions.argtypes = [vp]
    L.orc_num_nodes.restype = ctypes.c_long
    L.orc_num_nodes.argtypes = [vp]
    L.orc_num_markers.argtypes = [vp, ctypes.c_int]
    L.orc_error.argtypes = [vp]
    L.orc_get_populations.argtypes = [vp, dp, dp]
    L.orc_set_populations.argtypes = [vp, dp, dp]
    L.orc_get_particles.argtypes = [vp, dp]
    L.orc_set_particles.argtypes = [vp, dp]
    L.orc_get_reactions.argtypes = [vp, dp]
    L.orc_get_markers.argtypes = [vp, ctypes.c_int, dp]
    L.orc_fields.argtypes = [vp, dp, dp, dp, dp, dp]
    L.orc_totals.argtypes = [vp, dp]
    L.orc_raw_moments.argtypes = [vp, dp, dp, dp]
    L.orc_exchange.argtypes = [vp]
    L.orc_step_prescribed.argtypes = [vp, dp]
    L.orc_contacts.argtypes = [vp, ctypes.c_int, ip]
    L.orc_delta_h.restype = ctypes.c_double
    L.orc_delta_h.argtypes = [ctypes.c_double]
    L.orc_lagrange2.restype = ctypes.c_double
    L.orc_lagrange2.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_threads.argtypes = [ctypes.c_int]
    return L


def lib():
    """The oracle library built next to its source."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def derive(cfg: dict) -> dict:
    """Relaxation times and g*beta from the configuration (see module doc)."""
    dim = cfg["dim"]
    csg2 = 1.0 / 3.0 if dim == 2 or int(cfg.get("thermal_model", 0)) == 1 else 0.25
    if cfg.get("Ra", 0.0) > 0:
        Ra, Pr, Lc, uc = cfg["Ra"], cfg["Pr"], cfg["Lc"], cfg["uc"]
        nu = math.sqrt(Pr) * Lc * uc / math.sqrt(Ra)
        alpha = Lc * uc / math.sqrt(Pr * Ra)
        gbeta = uc * uc / (Lc * cfg.get("dT_ref", 1.0))
    else:
        nu = cfg["nu"]
        alpha = nu / cfg["Pr"]
        gbeta = cfg.get("Gr", 0.0) * nu * nu / cfg["Lc"] ** 3
    out = {"nu": nu, "alpha": alpha, "tau_f": 3.0 * nu + 0.5, "tau_g": alpha / csg2 + 0.5, "gbeta": gbeta}
    if cfg.get("tau_f", 0) > 0:
        out["tau_f"] = cfg["tau_f"]
        out["nu"] = (cfg["tau_f"] - 0.5) / 3.0
    if cfg.get("tau_g", 0) > 0:
        out["tau_g"] = cfg["tau_g"]
        out["alpha"] = (cfg["tau_g"] - 0.5) * csg2
    if "gbeta" in cfg and cfg["gbeta"] is not None:
        out["gbeta"] = cfg["gbeta"]
    return out


def make_params(cfg: dict) -> OrcParams:
    d = derive(cfg)
    p = OrcParams()
    p.dim = cfg["dim"]
    p.nx, p.ny = cfg["nx"], cfg["ny"]
    p.nz = cfg.get("nz", 1) if cfg["dim"] == 3 else 1
    per = cfg.get("periodic", [0, 0, 0])
    for i in range(3):
        p.periodic[i] = int(per[i])
    tw = cfg.get("T_wall", [0.0] * 6)
    for i in range(6):
        p.T_wall[i] = float(tw[i])
    p.T_init = cfg.get("T_init", 0.0)
    p.T_ref = cfg.get("T_ref", 0.0)
    p.tau_f, p.tau_g, p.gbeta = d["tau_f"], d["tau_g"], d["gbeta"]
    p.gravity = cfg.get("gravity", 0.0)
    p.kappa_T = cfg.get("kappa_T", 1.0)
    p.E_star = cfg.get("E_star", 0.0)
    p.poisson = cfg.get("poisson", 0.33)
    p.mu_fric = cfg.get("mu_fric", 0.3)
    p.n_sub = int(cfg.get("n_sub", 1))
    p.beta_p = cfg.get("beta_p", 0.0)
    p.c_r = cfg.get("c_r", 1.0)
    p.marker_mode = int(cfg.get("marker_mode", 0))
    p.interp_order = int(cfg.get("interp_order", 2))
    p.lattice = int(cfg.get("lattice", 19))
    p.thermal_model = int(cfg.get("thermal_model", 0))
    p.marker_spacing = cfg.get("marker_spacing", 1.0)
    return p


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """One FP64 simulation.  ``particles`` is an (n, 13) array:
    x[3] u[3] omega[3] R rho_r T flags (flags: 1 fixed, 2 thermosensitive)."""

    def __init__(self, cfg: dict, particles=None, library=None):
        self._L = library if library is not None else lib()
        self.cfg = dict(cfg)
        self.derived = derive(cfg)
        self.params = make_params(cfg)
        P = np.zeros((0, 13)) if particles is None else np.ascontiguousarray(particles, dtype=np.float64)
        self.np = P.shape[0]
        L = self._L
        self._h = L.orc_create(ctypes.byref(self.params), self.np, _dp(P) if self.np else None)
        self.dim = self.params.dim
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = int(L.orc_num_nodes(self._h))
        self.Q = 9 if self.dim == 2 else (15 if int(cfg.get("lattice", 19)) == 15 else 19)
        self.Qg = self.Q if int(cfg.get("thermal_model", 0)) == 1 else (5 if self.dim == 2 else 7)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        self._L.orc_step(self._h, int(n))

    def dem_only(self, n: int = 1):
        self._L.orc_dem_only(self._h, int(n))

    def clear_reactions(self):
        self._L.orc_clear_reactions(self._h)

    @property
    def error(self) -> int:
        return self._L.orc_error(self._h)

    def populations(self):
        f = np.empty((self.Q, self.N))
        g = np.empty((self.Qg, self.N))
        self._L.orc_get_populations(self._h, _dp(f), _dp(g))
        return f, g

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, self.N)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.Qg, self.N)
        self._L.orc_set_populations(self._h, _dp(f), _dp(g))

    def particles(self):
        out = np.empty((self.np, 16))
        if self.np:
            self._L.orc_get_particles(self._h, _dp(out))
        return out

    def set_particles(self, P):
        P = np.ascontiguousarray(P, dtype=np.float64)
        self._L.orc_set_particles(self._h, _dp(P))

    def reactions(self):
        out = np.empty((self.np, 8))
        if self.np:
            self._L.orc_get_reactions(self._h, _dp(out))
        return out

    def markers(self, i: int):
        n = self._L.orc_num_markers(self._h, i)
        out = np.empty((n, 4))
        self._L.orc_get_markers(self._h, i, _dp(out))
        return out

    def fields(self, forcing: bool = False):
        """rho (nz,ny,nx), u (nz,ny,nx,3), T (nz,ny,nx) of the next collision."""
        rho = np.empty(self.N)
        u = np.empty(self.N * 3)
        T = np.empty(self.N)
        FB = np.empty(self.N * 3) if forcing else None
        QB = np.empty(self.N) if forcing else None
        self._L.orc_fields(self._h, _dp(rho), _dp(u), _dp(T),
                         _dp(FB) if forcing else None, _dp(QB) if forcing else None)
        out = (rho.reshape(self.shape), u.reshape(self.shape + (3,)), T.reshape(self.shape))
        if forcing:
            out = out + (FB.reshape(self.shape + (3,)), QB.reshape(self.shape))
        return out

    def raw_moments(self):
        """Post-stream rho (N), j (N, 3), S (N) of the current state."""
        rho, j, S = np.empty(self.N), np.empty(3 * self.N), np.empty(self.N)
        self._L.orc_raw_moments(self._h, _dp(rho), _dp(j), _dp(S))
        return rho, j.reshape(self.N, 3), S

    def step_prescribed(self, FH):
        """One one-point step with prescribed reactions FH (n, 4): the force
        on each particle and the heat it gives the fluid, in place of the
        Lagrangian-point exchange."""
        FH = np.ascontiguousarray(FH, dtype=np.float64).reshape(self.np, 4)
        self._L.orc_step_prescribed(self._h, _dp(FH))

    def exchange(self):
        """Evaluate the point exchange on the current state; its reactions
        become what reactions() returns."""
        self._L.orc_exchange(self._h)

    def totals(self):
        out = np.empty(5)
        self._L.orc_totals(self._h, _dp(out))
        return out

    def contacts(self, i: int):
        buf = (ctypes.c_int * max(self.np, 1))()
        n = self._L.orc_contacts(self._h, i, buf)
        return [buf[k] for k in range(n)]


def delta_h(a: float) -> float:
    return lib().orc_delta_h(float(a))


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().orc_set_threads(int(n))
