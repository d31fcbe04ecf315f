"""Seeded input generators: reproducible, non-overlapping, inside the box."""
import numpy as np
import pytest

from paper_1502_01159_amd import workloads as W


def test_splitmix64_reference_values():
    """splitmix64 from seed 0 (published generator; first outputs)."""
    g = W.SplitMix64(0)
    assert g.next_u64() == 0xE220A8397B1DCDAF
    assert g.next_u64() == 0x6E789E6AA1B965F4
    assert g.next_u64() == 0x06C45D188009454F


def _check(cfg, P):
    d = cfg["dim"]
    n = [cfg["nx"], cfg["ny"], cfg.get("nz", 1)]
    X = P[:, :d]
    R = P[:, 9]
    for a in range(d):
        assert np.all(X[:, a] - R >= -0.5) and np.all(X[:, a] + R <= n[a] - 0.5)
    from scipy.spatial import cKDTree
    t = cKDTree(X)
    pairs = t.query_pairs(2 * R.max() - 1e-9)
    for i, j in pairs:
        assert np.linalg.norm(X[i] - X[j]) >= R[i] + R[j] - 1e-9


@pytest.mark.parametrize("name", ["c1", "c2", "c2_small", "c3_small", "c3_mid", "c4_small", "c4_mid", "c3", "c4", "x2"])
def test_workloads_valid_and_reproducible(name):
    cfg, P = W.workload(name)
    _check(cfg, P)
    cfg2, P2 = W.workload(name)
    assert np.array_equal(P, P2)


def test_full_sizes():
    cfg, P = W.workload("c3")
    assert (cfg["nx"], cfg["ny"], cfg["nz"], len(P)) == (256, 256, 512, 2000)
    assert np.all(P[:, 9] == 6.0) and np.all(P[:, 10] == 1.05)
    cfg, P = W.workload("c4")
    assert (cfg["nx"], len(P)) == (384, 20000)
    # density ratio 1.25, with (rho_r - 1) g that of the heated spheres above
    assert np.all(P[:, 10] == 1.25)
    assert abs((1.25 - 1.0) * cfg["gravity"] - 0.05 * W.workload("c3")[0]["gravity"]) < 1e-12
    assert np.all(P[:, 12] == W.THERMO)
    assert 0.0 <= P[:, 11].min() and P[:, 11].max() < 1.0
    cfg, P = W.workload("c2")
    assert (cfg["nx"], cfg["ny"], len(P)) == (512, 1024, 100)
