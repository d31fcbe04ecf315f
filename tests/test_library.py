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
