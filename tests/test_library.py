"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/pibm.h declares, and its host-side planning validates parameters.
No compute call is made (no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1502_01159_amd import pibm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pibm.h")).read()
    return sorted(set(re.findall(r"\b(pibm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pibm.LIB_PATH):
        from paper_1502_01159_amd import build as B
        B.build()
    return pibm.lib()


def test_exports_match_header(L):
    names = _declared()
    assert set(names) == set(pibm.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_workspace_bytes_and_validation(L):
    cfg, P = W.workload("c1")
    p = pibm.make_params(cfg)
    parts = pibm.make_particles(P)
    nb = L.pibm_workspace_bytes(ctypes.byref(p), parts, len(P))
    N = 64 * 64
    # at least both lattice copies (14 populations, 4 bytes)
    assert nb >= 2 * 14 * N * 4
    p64 = pibm.make_params(cfg, "f64")
    assert L.pibm_workspace_bytes(ctypes.byref(p64), parts, len(P)) > nb
    bad = pibm.make_params(dict(cfg, tau_f=0.5))        # tau must exceed 1/2
    assert L.pibm_workspace_bytes(ctypes.byref(bad), parts, len(P)) == 0
    bad = pibm.make_params(dict(cfg, dim=4))
    assert L.pibm_workspace_bytes(ctypes.byref(bad), parts, len(P)) == 0


def test_lattice_and_interpolation_options_validated(L):
    """D3Q15 is accepted in 3D with FP32/FP64 storage and sized for 15 + 7
    populations; D3Q15 in 2D or with 16-bit storage, and interpolation orders
    other than 2 and 4, are refused (the sizing call returns 0)."""
    cfg, P = W.workload("c3_small")
    parts = pibm.make_particles(P)
    size = lambda c, st="f32": L.pibm_workspace_bytes(ctypes.byref(pibm.make_params(c, st)), parts, len(P))
    n19, n15 = size(cfg), size(dict(cfg, lattice=15))
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    assert n15 > 0 and n19 - n15 >= 2 * 4 * N * 4          # four fewer flow populations, two copies
    assert size(dict(cfg, lattice=15), "f64") > 0
    assert size(dict(cfg, lattice=15), "f16") == 0
    assert size(dict(cfg, lattice=15), "bf16") == 0
    assert size(dict(cfg, lattice=17)) == 0
    c2, P2 = W.workload("c1")
    assert L.pibm_workspace_bytes(ctypes.byref(pibm.make_params(dict(c2, lattice=15))),
                                  pibm.make_particles(P2), len(P2)) == 0
    assert size(dict(cfg, interp_order=4)) > 0
    assert size(dict(cfg, interp_order=3)) == 0
    # temperature on the flow lattice: 19 + 19 populations, FP32 / FP64 only
    n_tm = size(dict(cfg, thermal_model=1))
    assert n_tm - n19 >= 2 * 12 * N * 4
    assert size(dict(cfg, thermal_model=1), "f64") > 0
    assert size(dict(cfg, thermal_model=1), "f16") == 0
    assert size(dict(cfg, thermal_model=2)) == 0
    # one or two streams: same workspace, other values refused
    assert size(dict(cfg, streams=1)) == size(dict(cfg, streams=2)) == n19
    assert size(dict(cfg, streams=3)) == 0 and size(dict(cfg, streams=-1)) == 0


def test_full_size_workspace_fits_hbm(L):
    """Every workload fits one MI355X (288 GB) with room to spare."""
    for name in ("c2", "c3", "c4"):
        cfg, P = W.workload(name)
        for st in ("f32", "f16", "f64"):
            p = pibm.make_params(cfg, st)
            nb = L.pibm_workspace_bytes(ctypes.byref(p), pibm.make_particles(P), len(P))
            assert 0 < nb < 100e9, (name, st, nb)


def test_init_rejects_bad_input_without_gpu(L):
    """pibm_init validates before touching the device."""
    cfg, P = W.workload("c2_small")
    p = pibm.make_params(cfg)
    h = ctypes.c_void_p()
    P2 = P.copy()
    P2[1, :3] = P2[0, :3] + 0.5               # overlapping pair
    parts = pibm.make_particles(P2)
    st = L.pibm_init(ctypes.byref(h), ctypes.byref(p), parts, len(P2), ctypes.c_void_p(256), 1 << 40, None)
    assert st == pibm.EOVERLAP
    P3 = P.copy()
    P3[0, 0] = -3.0                            # centre beyond the wall
    st = L.pibm_init(ctypes.byref(h), ctypes.byref(p), pibm.make_particles(P3), len(P3), ctypes.c_void_p(256),
                     1 << 40, None)
    assert st == pibm.EINVAL
    st = L.pibm_init(ctypes.byref(h), ctypes.byref(p), pibm.make_particles(P), len(P), ctypes.c_void_p(256), 16, None)
    assert st == pibm.EINVAL                   # workspace too small
    assert L.pibm_strerror(pibm.EOVERLAP).decode().startswith("initial particles")
