"""Pins of the FP64 closure-network oracle against the mathematics: the
GELU identities, the chain rule against central finite differences, a
network reduced to closed form, and Adam's first step."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1502_01159_amd import workloads as W


def params(seed, scale=1.0):
    rng = W.SplitMix64(seed)
    p = np.empty(M.NPARAM)
    k = 0
    for i, o in M.SIZES:
        lim = scale / math.sqrt(i)
        p[k:k + i * o] = (2.0 * rng.uniforms(i * o) - 1.0) * lim
        k += i * o
        p[k:k + o] = (2.0 * rng.uniforms(o) - 1.0) * 0.1
        k += o
    return p


def batch(seed, n):
    rng = W.SplitMix64(seed)
    x = (2.0 * rng.uniforms(n * 16) - 1.0).reshape(n, 16) * 2.0
    t = (2.0 * rng.uniforms(n * 4) - 1.0).reshape(n, 4)
    return x, t


def test_gelu_identities():
    """GELU(z) = z Phi(z): GELU(z) - GELU(-z) = z, GELU(0) = 0,
    GELU'(0) = 1/2, GELU(z) -> z for large z, Phi(1) from the erf table."""
    z = np.linspace(-6, 6, 121)
    assert np.allclose(M.gelu(z) - M.gelu(-z), z, rtol=0, atol=1e-15)
    assert M.gelu(0.0) == 0.0 and M.gelu_d(0.0) == 0.5
    assert M.gelu(8.0) == pytest.approx(8.0, abs=1e-14)
    assert M.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-15)   # Phi(1)
    h = 1e-6
    assert np.allclose(M.gelu_d(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), atol=1e-9)


def test_gradients_match_central_differences():
    """P14 (FP64 part): every parameter's analytic gradient against
    (L(p + h e) - L(p - h e)) / 2h on a small batch, h = 1e-6."""
    p = params(1)
    x, t = batch(2, 5)
    L, g = M.loss_and_grads(p, x, t)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(M.NPARAM, 300, replace=False),
                          [0, 2047, 2048 + 127, M.NPARAM - 5, M.NPARAM - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss_and_grads(p + e, x, t)[0] - M.loss_and_grads(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_constant_network_closed_form():
    """With every weight zero the output is b4; the loss gradient on b4 is
    (b4 - mean t) / 2 and every other gradient vanishes except the last
    layer's weights, whose inputs are GELU(b3)."""
    p = np.zeros(M.NPARAM)
    layers = M.unpack(p)
    layers[3][1][:] = [0.5, -1.0, 0.25, 2.0]
    layers[2][1][:] = 0.3
    x, t = batch(3, 7)
    L, g = M.loss_and_grads(p, x, t)
    y = np.array([0.5, -1.0, 0.25, 2.0])
    assert L == pytest.approx(((y - t) ** 2).sum() / (4 * 7), rel=1e-14)
    gl = M.unpack(g)
    assert np.allclose(gl[3][1], (y - t.mean(0)) / 2, rtol=1e-14)
    assert np.allclose(gl[3][0], M.gelu(0.3) * np.tile((y - t.mean(0)) / 2, (128, 1)), rtol=1e-13)
    for l in range(3):
        assert not gl[l][0].any() and not gl[l][1].any()


def test_adam_first_step_is_sign_step():
    """Adam's bias-corrected first step moves every parameter by
    lr g / (|g| + eps), i.e. lr sign(g) for |g| >> eps."""
    p = params(4)
    g = np.linspace(-1, 1, M.NPARAM) + 1e-3
    opt = M.Adam(p, lr=1e-3)
    p1 = opt.step(g)
    assert np.allclose(p1 - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_bf16_rounding_reference_values():
    """Round to nearest even at 8 mantissa bits: 1 + 2^-8 (a tie) stays 1,
    1 + 3 * 2^-8 rounds up to 1 + 2^-6, 1 + 2^-7 is exact."""
    v = M.bf16(np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -3.0, 0.0]))
    assert list(v) == [1.0, 1 + 2 ** -6, 1 + 2 ** -7, -3.0, 0.0]
