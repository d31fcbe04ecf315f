"""Pins of the closure-feature reference against closed forms: uniform
fields give the slip, Reynolds and Grashof numbers exactly; a known
arrangement gives the solid fraction and the neighbour offsets."""
import math

import numpy as np
import pytest

from oracle import closure_oracle as C


def prow(x, u, R, T):
    r = np.zeros(16)
    r[0:3], r[3:6], r[12], r[14] = x, u, R, T
    return r


def test_uniform_flow_features_closed_form():
    """A uniform field gives the slip, Re_p, Gr_p and T_p - T_f exactly."""
    shape = (24, 20, 28)
    N = int(np.prod(shape))
    u0 = np.array([0.02, -0.01, 0.005])
    rho = np.full(N, 1.1)
    j = np.tile(rho[:, None] * u0, (1, 1))
    S = np.full(N, 0.3)
    P = np.array([prow((10.3, 9.7, 12.2), (0.0, 0.01, 0.0), 2.0, 0.8),
                  prow((17.0, 9.7, 12.2), (0.0, 0.0, 0.0), 2.0, 0.8)])
    nu, gb = 0.05, 1e-4
    for _ in range(1):
        X, s, Tf = C.features(rho, j, S, shape, [1, 1, 1], P, nu, gb, 3)
        slip = u0 - P[0, 3:6]
        assert np.allclose(s[0], slip, rtol=1e-12)
        assert Tf[0] == pytest.approx(0.3, rel=1e-13)
        assert X[0, 0] == pytest.approx(np.linalg.norm(slip) * 4.0 / nu, rel=1e-12)
        assert X[0, 1] == pytest.approx(gb * 0.5 * 64.0 / nu ** 2, rel=1e-12)
        assert X[0, 3] == pytest.approx(0.5, rel=1e-13)
        # the neighbour at +6.7 x lies at 6.7/4 along x, seen in the slip frame
        e1, e2, e3 = C.slip_frame(slip, 3)
        d = np.array([6.7, 0.0, 0.0]) / 4.0
        assert np.allclose(X[0, 4:7], [d.dot(e1), d.dot(e2), d.dot(e3)], rtol=1e-12)
        assert np.allclose(X[0, 7:16], 4.0)           # no further neighbours
        # both centres are within 2D = 8 of each other: phi = 2 spheres / ball
        assert X[0, 2] == pytest.approx(2 * (4 / 3) * math.pi * 8 / ((4 / 3) * math.pi * 512), rel=1e-12)


def test_frame_is_orthonormal_and_right_handed():
    rng = np.random.default_rng(0)
    for _ in range(50):
        s = rng.normal(size=3)
        e1, e2, e3 = C.slip_frame(s, 3)
        M = np.array([e1, e2, e3])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(M) == pytest.approx(1.0, abs=1e-13)
        assert np.allclose(e1, s / np.linalg.norm(s))
    e1, e2, e3 = C.slip_frame(np.array([0.0, 0.0, -2.0]), 3)    # vertical slip: e2 from x
    assert np.allclose(e2, [1, 0, 0]) and np.allclose(e3, np.cross(e1, e2))


def test_targets_roundtrip_frame():
    rng = np.random.default_rng(1)
    F = rng.normal(size=(5, 3))
    H = rng.normal(size=5)
    s = rng.normal(size=(5, 3))
    R = np.full(5, 3.0)
    dT = rng.uniform(0.1, 1.0, 5)
    t = C.targets(F, H, s, R, dT, 0.1, 0.05, 3)
    for p in range(5):
        e1, e2, e3 = C.slip_frame(s[p], 3)
        fs = 3 * math.pi * 0.1 * 6.0 * np.linalg.norm(s[p])
        assert np.allclose(fs * (t[p, 0] * e1 + t[p, 1] * e2 + t[p, 2] * e3), F[p], rtol=1e-12)
        assert t[p, 3] == pytest.approx(H[p] / (math.pi * 6.0 * 0.05 * dT[p]), rel=1e-13)
    # Stokes drag along the slip has drag factor 1; zero slip gives zeros
    t1 = C.targets(np.array([[0.0, 0.0, 3 * math.pi * 0.1 * 6.0 * 0.02]]), np.zeros(1),
                   np.array([[0.0, 0.0, 0.02]]), np.array([3.0]), np.array([1.0]), 0.1, 0.05, 3)
    assert t1[0, 0] == pytest.approx(1.0, rel=1e-14) and t1[0, 3] == 0.0
    t0 = C.targets(F[:1], H[:1], np.zeros((1, 3)), R[:1], np.zeros(1), 0.1, 0.05, 3)
    assert not t0.any()
