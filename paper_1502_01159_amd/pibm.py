"""ctypes binding of the C ABI in ``include/pibm.h`` (``libpibm.so``).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch provides the device workspace and the stream.  When the
library is missing the import still works (so that CPU-only tools can read the
configuration helpers) but creating a :class:`Simulation` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpibm.so")

STORAGE = {"f32": 0, "f64": 1, "f16": 2, "bf16": 3}
MARKERS = {"surface": 0, "paper": 1, "point": 2}

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, EOVERLAP, ESTATE = 0, -1, -2, -3, -4, -5, -6

EXPORTS = [
    "pibm_workspace_bytes", "pibm_init", "pibm_step", "pibm_sync", "pibm_particles", "pibm_set_particles",
    "pibm_fields", "pibm_get_populations", "pibm_set_populations", "pibm_num_nodes", "pibm_num_markers",
    "pibm_step_count", "pibm_derived", "pibm_save", "pibm_load", "pibm_destroy", "pibm_strerror",
    "pibm_profile", "pibm_profile_phases", "pibm_profile_read",
    "pibm_mlp_workspace_bytes", "pibm_mlp_create", "pibm_mlp_set_params", "pibm_mlp_get_params",
    "pibm_mlp_forward", "pibm_mlp_grads", "pibm_mlp_train_step", "pibm_mlp_destroy",
    "pibm_features", "pibm_set_closure", "pibm_mlp_grads_noalloc", "pibm_set_closure_range",
]
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_NPARAM = 16, 128, 4, 35716
MLP_NOALLOC_MAX_BATCH = 4096
PHASES = ("markers", "bin", "lattice", "dem")


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("periodic", ctypes.c_int * 3), ("storage", ctypes.c_int),
        ("T_wall", ctypes.c_double * 6), ("T_init", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("Lc", ctypes.c_double), ("uc", ctypes.c_double),
        ("dT_ref", ctypes.c_double), ("nu", ctypes.c_double), ("Gr", ctypes.c_double),
        ("tau_f", ctypes.c_double), ("tau_g", ctypes.c_double), ("gbeta", ctypes.c_double),
        ("gbeta_set", ctypes.c_int), ("marker_mode", ctypes.c_int), ("marker_spacing", ctypes.c_double),
        ("gravity", ctypes.c_double), ("kappa_T", ctypes.c_double), ("E_star", ctypes.c_double),
        ("poisson", ctypes.c_double), ("mu_fric", ctypes.c_double), ("n_sub", ctypes.c_int),
        ("beta_p", ctypes.c_double), ("c_r", ctypes.c_double), ("skin", ctypes.c_double),
        ("interp_order", ctypes.c_int), ("lattice", ctypes.c_int), ("thermal_model", ctypes.c_int),
        ("streams", ctypes.c_int),
    ]


class Particle(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_double * 3), ("u", ctypes.c_double * 3), ("omega", ctypes.c_double * 3),
        ("theta", ctypes.c_double * 3), ("R", ctypes.c_double), ("rho_r", ctypes.c_double),
        ("T", ctypes.c_double), ("flags", ctypes.c_int), ("reserved", ctypes.c_int),
    ]


class PibmError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


_lib = None


def lib():
    """Load libpibm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        PP = ctypes.POINTER(Particle)
        L.pibm_workspace_bytes.restype = sz
        L.pibm_workspace_bytes.argtypes = [ctypes.POINTER(Params), PP, ctypes.c_int]
        L.pibm_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Params), PP, ctypes.c_int, vp, sz, vp]
        L.pibm_step.argtypes = [vp, ctypes.c_int]
        L.pibm_sync.argtypes = [vp]
        L.pibm_particles.argtypes = [vp, PP, dp, ctypes.c_int]
        L.pibm_set_particles.argtypes = [vp, PP, ctypes.c_int]
        L.pibm_fields.argtypes = [vp, dp, dp, dp]
        L.pibm_get_populations.argtypes = [vp, dp, dp]
        L.pibm_set_populations.argtypes = [vp, dp, dp]
        for f in ("pibm_num_nodes", "pibm_num_markers", "pibm_step_count"):
            getattr(L, f).restype = ctypes.c_longlong
            getattr(L, f).argtypes = [vp]
        L.pibm_derived.argtypes = [vp, dp]
        L.pibm_save.argtypes = [vp, vp, sz, ctypes.POINTER(sz)]
        L.pibm_load.argtypes = [vp, vp, sz]
        L.pibm_destroy.argtypes = [vp]
        L.pibm_profile.argtypes = [vp, ctypes.c_int]
        L.pibm_profile_phases.argtypes = [vp, ctypes.c_uint]
        L.pibm_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong)]
        L.pibm_strerror.restype = ctypes.c_char_p
        L.pibm_strerror.argtypes = [ctypes.c_int]
        fp = ctypes.POINTER(ctypes.c_float)
        L.pibm_mlp_workspace_bytes.restype = sz
        L.pibm_mlp_workspace_bytes.argtypes = [ctypes.c_int]
        L.pibm_mlp_create.argtypes = [ctypes.POINTER(vp), ctypes.c_ulonglong, ctypes.c_int, vp, sz, vp]
        L.pibm_mlp_set_params.argtypes = [vp, fp]
        L.pibm_mlp_get_params.argtypes = [vp, fp]
        L.pibm_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int]
        L.pibm_mlp_grads.argtypes = [vp, vp, vp, ctypes.c_int, fp, dp]
        L.pibm_mlp_grads_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, fp, dp]
        L.pibm_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_float, dp]
        L.pibm_mlp_destroy.argtypes = [vp]
        L.pibm_features.argtypes = [vp, fp, fp]
        L.pibm_set_closure.argtypes = [vp, vp, fp]
        L.pibm_set_closure_range.argtypes = [vp, fp, fp]
        _lib = L
    return _lib


def strerror(status: int) -> str:
    try:
        return lib().pibm_strerror(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def make_params(cfg: dict, storage: str = "f32") -> Params:
    p = Params()
    p.dim = int(cfg["dim"])
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.nz = int(cfg.get("nz", 1)) if p.dim == 3 else 1
    per = cfg.get("periodic", [0, 0, 0])
    for i in range(3):
        p.periodic[i] = int(per[i])
    p.storage = STORAGE[storage]
    tw = cfg.get("T_wall", [0.0] * 6)
    for i in range(6):
        p.T_wall[i] = float(tw[i])
    p.T_init = float(cfg.get("T_init", 0.0))
    p.T_ref = float(cfg.get("T_ref", 0.0))
    for k in ("Ra", "Pr", "Lc", "uc", "nu", "Gr"):
        setattr(p, k, float(cfg.get(k, 0.0)))
    p.dT_ref = float(cfg.get("dT_ref", 1.0))
    p.tau_f = float(cfg.get("tau_f", 0.0))
    p.tau_g = float(cfg.get("tau_g", 0.0))
    if cfg.get("gbeta") is not None:
        p.gbeta, p.gbeta_set = float(cfg["gbeta"]), 1
    p.marker_mode = int(cfg.get("marker_mode", 1))
    p.marker_spacing = float(cfg.get("marker_spacing", 1.0))
    p.gravity = float(cfg.get("gravity", 0.0))
    p.kappa_T = float(cfg.get("kappa_T", 1.0))
    p.E_star = float(cfg.get("E_star", 0.0))
    p.poisson = float(cfg.get("poisson", 0.33))
    p.mu_fric = float(cfg.get("mu_fric", 0.3))
    p.n_sub = int(cfg.get("n_sub", 1))
    p.beta_p = float(cfg.get("beta_p", 0.0))
    p.c_r = float(cfg.get("c_r", 1.0))
    p.skin = float(cfg.get("skin", 1.0))
    p.interp_order = int(cfg.get("interp_order", 2))
    p.lattice = int(cfg.get("lattice", 19))
    p.thermal_model = int(cfg.get("thermal_model", 0))
    p.streams = int(cfg.get("streams", 0))
    return p


def make_particles(P) -> ctypes.Array:
    """(n, 13) rows x[3] u[3] omega[3] R rho_r T flags -> pibm_particle[n]."""
    P = np.zeros((0, 13)) if P is None else np.asarray(P, dtype=np.float64)
    arr = (Particle * max(len(P), 1))()
    for i, r in enumerate(P):
        q = arr[i]
        for k in range(3):
            q.x[k], q.u[k], q.omega[k], q.theta[k] = r[k], r[3 + k], r[6 + k], 0.0
        q.R, q.rho_r, q.T, q.flags = r[9], r[10], r[11], int(r[12])
    return arr


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Simulation:
    """One simulation on one GPU through the C ABI.

    ``cfg``/``particles`` follow :mod:`paper_1502_01159_amd.workloads`.  The
    workspace is a torch uint8 tensor on ``device``; all work is queued on
    ``stream`` (default: torch's current stream of that device)."""

    def __init__(self, cfg: dict, particles=None, storage: str = "f32", device: str = "cuda:0", stream=None):
        import torch

        L = lib()
        self.cfg = dict(cfg)
        self.storage = storage
        self.params = make_params(cfg, storage)
        P = np.zeros((0, 13)) if particles is None else np.asarray(particles, dtype=np.float64)
        self.np = len(P)
        self._parts = make_particles(P)
        self.device = torch.device(device)
        nbytes = L.pibm_workspace_bytes(ctypes.byref(self.params), self._parts, self.np)
        if nbytes == 0:
            raise PibmError(EINVAL, "pibm_workspace_bytes")
        self.workspace_bytes = int(nbytes)
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = ctypes.c_void_p()
        st = L.pibm_init(ctypes.byref(self._h), ctypes.byref(self.params), self._parts, self.np,
                         ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(self.workspace_bytes),
                         ctypes.c_void_p(self._stream.cuda_stream))
        if st != OK:
            raise PibmError(st, "pibm_init")
        self.dim = self.params.dim
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = int(L.pibm_num_nodes(self._h))
        self.Q = 9 if self.dim == 2 else (15 if int(cfg.get("lattice", 19)) == 15 else 19)
        self.Qg = self.Q if int(cfg.get("thermal_model", 0)) == 1 else (5 if self.dim == 2 else 7)
        d = np.empty(5)
        L.pibm_derived(self._h, _dp(d))
        self.derived = dict(tau_f=d[0], tau_g=d[1], gbeta=d[2], nu=d[3], alpha=d[4])

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().pibm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != OK:
            raise PibmError(st, what)

    # -- stepping ----------------------------------------------------------
    def step(self, n: int = 1):
        self._check(lib().pibm_step(self._h, int(n)), "pibm_step")

    def sync(self) -> int:
        return lib().pibm_sync(self._h)

    @property
    def num_markers(self) -> int:
        return int(lib().pibm_num_markers(self._h))

    @property
    def step_count(self) -> int:
        return int(lib().pibm_step_count(self._h))

    # -- state access ------------------------------------------------------
    def particles(self, check: bool = True):
        """(n, 16) rows x[3] u[3] omega[3] theta[3] R rho_r T flags, and the
        (n, 8) reactions F[3] tau[3] H sum (T_p - T_l) A_l."""
        arr = (Particle * max(self.np, 1))()
        fth = np.empty((max(self.np, 1), 8))
        st = lib().pibm_particles(self._h, arr, _dp(fth), max(self.np, 1))
        if check:
            self._check(st, "pibm_particles")
        out = np.empty((self.np, 16))
        for i in range(self.np):
            q = arr[i]
            out[i, 0:3], out[i, 3:6], out[i, 6:9], out[i, 9:12] = q.x[:], q.u[:], q.omega[:], q.theta[:]
            out[i, 12], out[i, 13], out[i, 14], out[i, 15] = q.R, q.rho_r, q.T, q.flags
        return out, fth[: self.np]

    def set_particles(self, P):
        arr = make_particles(P)
        self._check(lib().pibm_set_particles(self._h, arr, len(P)), "pibm_set_particles")

    def features(self):
        """Closure features (n, 16) and targets (n, 4) of the current state."""
        x = np.empty((self.np, 16), dtype=np.float32)
        t = np.empty((self.np, 4), dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        st = lib().pibm_features(self._h, x.ctypes.data_as(fp), t.ctypes.data_as(fp))
        if st != OK:
            raise PibmError(st, "pibm_features")
        return x, t

    def set_closure(self, mlp, norm=None):
        """Use the network `mlp` (an :class:`Mlp`) in the one-point mode;
        norm = 40 floats (feature mean, std, target mean, std).  None restores
        the point exchange."""
        if mlp is None:
            st = lib().pibm_set_closure(self._h, None, None)
        else:
            norm = np.ascontiguousarray(norm, dtype=np.float32)
            if norm.size != 40:
                raise ValueError("norm must hold 40 values")
            self._closure = (mlp, norm)
            st = lib().pibm_set_closure(self._h, mlp._h, norm.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        if st != OK:
            raise PibmError(st, "pibm_set_closure")

    def set_closure_range(self, lo, hi):
        """Particles whose 16 raw features (as :meth:`features` returns them)
        leave [lo, hi] keep the point exchange; None, None removes the range."""
        fp = ctypes.POINTER(ctypes.c_float)
        if lo is None and hi is None:
            st = lib().pibm_set_closure_range(self._h, None, None)
        else:
            lo = np.ascontiguousarray(lo, dtype=np.float32)
            hi = np.ascontiguousarray(hi, dtype=np.float32)
            if lo.size != 16 or hi.size != 16:
                raise ValueError("lo and hi must hold 16 values each")
            self._range = (lo, hi)
            st = lib().pibm_set_closure_range(self._h, lo.ctypes.data_as(fp), hi.ctypes.data_as(fp))
        if st != OK:
            raise PibmError(st, "pibm_set_closure_range")

    def fields(self, check: bool = True):
        rho = np.empty(self.N)
        u = np.empty(3 * self.N)
        T = np.empty(self.N)
        st = lib().pibm_fields(self._h, _dp(rho), _dp(u), _dp(T))
        if check:
            self._check(st, "pibm_fields")
        return rho.reshape(self.shape), u.reshape(self.shape + (3,)), T.reshape(self.shape)

    def populations(self):
        f = np.empty((self.Q, self.N))
        g = np.empty((self.Qg, self.N))
        self._check(lib().pibm_get_populations(self._h, _dp(f), _dp(g)), "pibm_get_populations")
        return f, g

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, self.N)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(self.Qg, self.N)
        self._check(lib().pibm_set_populations(self._h, _dp(f), _dp(g)), "pibm_set_populations")

    def profile(self, enable: bool = True, phases=None):
        """Time every phase (or none); `phases` (names from PHASES) times only
        those, since each timed phase adds a pair of events to the stream."""
        if phases is None:
            self._check(lib().pibm_profile(self._h, int(bool(enable))), "pibm_profile")
            return
        mask = 0
        for p in phases:
            mask |= 1 << PHASES.index(p)
        self._check(lib().pibm_profile_phases(self._h, mask if enable else 0), "pibm_profile_phases")

    def profile_read(self) -> dict:
        """{phase: (total ms, timed executions)} since the previous read."""
        ms = np.zeros(len(PHASES))
        cnt = (ctypes.c_longlong * len(PHASES))()
        self._check(lib().pibm_profile_read(self._h, _dp(ms), cnt), "pibm_profile_read")
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(PHASES)}

    def save(self) -> bytes:
        used = ctypes.c_size_t()
        self._check(lib().pibm_save(self._h, None, 0, ctypes.byref(used)), "pibm_save")
        buf = ctypes.create_string_buffer(used.value)
        self._check(lib().pibm_save(self._h, buf, used, ctypes.byref(used)), "pibm_save")
        return buf.raw

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(lib().pibm_load(self._h, buf, len(blob)), "pibm_load")


class Mlp:
    """The closure network (``pibm_mlp_*``) on the current CUDA device.

    Inputs are torch tensors on the device: ``x`` of shape (n, 16) and dtype
    bfloat16, targets ``t`` of shape (n, 4) float32.  Parameters are numpy
    float32 vectors in the canonical order of ``include/pibm.h``."""

    def __init__(self, seed: int = 0, max_batch: int = 4096):
        import torch

        L = lib()
        self._torch = torch
        nbytes = L.pibm_mlp_workspace_bytes(int(max_batch))
        if nbytes == 0:
            raise PibmError(EINVAL, "pibm_mlp_workspace_bytes")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        st = L.pibm_mlp_create(ctypes.byref(h), int(seed), int(max_batch), ctypes.c_void_p(aligned),
                               nbytes, ctypes.c_void_p(self._stream))
        if st != OK:
            raise PibmError(st, "pibm_mlp_create")
        self._h = h
        self.max_batch = int(max_batch)

    @staticmethod
    def _check(x, t=None):
        import torch

        if x.dtype != torch.bfloat16 or x.dim() != 2 or x.shape[1] != MLP_IN or not x.is_contiguous() or not x.is_cuda:
            raise ValueError("x must be a contiguous CUDA bfloat16 tensor of shape (n, 16)")
        if t is not None and (t.dtype != torch.float32 or tuple(t.shape) != (x.shape[0], MLP_OUT)
                              or not t.is_contiguous() or not t.is_cuda):
            raise ValueError("t must be a contiguous CUDA float32 tensor of shape (n, 4)")

    def get_params(self) -> np.ndarray:
        out = np.empty(MLP_NPARAM, dtype=np.float32)
        st = lib().pibm_mlp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        if st != OK:
            raise PibmError(st, "pibm_mlp_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != MLP_NPARAM:
            raise ValueError("wrong parameter count")
        st = lib().pibm_mlp_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        if st != OK:
            raise PibmError(st, "pibm_mlp_set_params")

    def forward(self, x, y=None):
        self._check(x)
        if y is None:
            y = self._torch.empty((x.shape[0], MLP_OUT), dtype=self._torch.float32, device=x.device)
        st = lib().pibm_mlp_forward(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.shape[0])
        if st != OK:
            raise PibmError(st, "pibm_mlp_forward")
        return y

    def grads(self, x, t):
        self._check(x, t)
        g = np.empty(MLP_NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        st = lib().pibm_mlp_grads(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()), x.shape[0],
                                  g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss))
        if st != OK:
            raise PibmError(st, "pibm_mlp_grads")
        return loss.value, g

    def grads_noalloc(self, x, t):
        """As :meth:`grads`, through the allocation-free entry point (batch up
        to ``MLP_NOALLOC_MAX_BATCH`` whatever this network's ``max_batch``)."""
        self._check(x, t)
        g = np.empty(MLP_NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        st = lib().pibm_mlp_grads_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                          x.shape[0], g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          ctypes.byref(loss))
        if st != OK:
            raise PibmError(st, "pibm_mlp_grads_noalloc")
        return loss.value, g

    def train_step(self, x, t, lr: float) -> float:
        self._check(x, t)
        loss = ctypes.c_double()
        st = lib().pibm_mlp_train_step(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                       x.shape[0], float(lr), ctypes.byref(loss))
        if st != OK:
            raise PibmError(st, "pibm_mlp_train_step")
        return loss.value

    def close(self):
        if getattr(self, "_h", None):
            lib().pibm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
