"""FP64 CPU oracle of the learned per-particle closure network.

TEST INFRASTRUCTURE ONLY: the plain reference that the GPU network is
checked against.  Only tests/, the smoke check and the benchmark's CPU
baseline may import it; it shares no code with the HIP library.

Network: 16 -> 128 -> 128 -> 128 -> 4, z = h W + b per layer, GELU(z) =
z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 on the hidden layers, identity output.
Loss of a batch of n samples: L = sum_s sum_c (y_sc - t_sc)^2 / (4 n).
Optimiser: Adam (Kingma & Ba 2015) with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8 and bias correction.

Parameters are one flat vector in the order W1[16][128], b1[128],
W2[128][128], b2[128], W3[128][128], b3[128], W4[128][4], b4[4].

`mirror=True` evaluates the same formulas but rounds to bfloat16 (round to
nearest even, through float32) where the GPU kernels feed a matrix-core
product: inputs, weights, hidden activations, the output gradient and the
pre-activation gradients; bias gradients are then sums of the rounded
pre-activation gradients.  Everything else stays FP64.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SIZES = [(16, 128), (128, 128), (128, 128), (128, 4)]
NPARAM = sum(i * o + o for i, o in SIZES)


def unpack(p):
    """Flat parameters -> [(W, b)] per layer (views)."""
    out, k = [], 0
    for i, o in SIZES:
        W = p[k:k + i * o].reshape(i, o)
        k += i * o
        b = p[k:k + o]
        k += o
        out.append((W, b))
    return out


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) through float32; float64 out."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(p, x, mirror=False, keep=False):
    """y[n][4] for inputs x[n][16]; with keep, also the per-layer (input,
    pre-activation) pairs the backward pass needs."""
    q = bf16 if mirror else (lambda a: np.asarray(a, dtype=np.float64))
    h = q(x)
    saved = []
    layers = unpack(np.asarray(p, dtype=np.float64))
    for l, (W, b) in enumerate(layers):
        z = h @ q(W) + b
        saved.append((h, z))
        if l < 3:
            h = q(gelu(z))
    return (z, saved) if keep else z


def loss_and_grads(p, x, t, mirror=False):
    """Loss L and dL/dparam (flat, canonical order), by the chain rule."""
    q = bf16 if mirror else (lambda a: np.asarray(a, dtype=np.float64))
    n = x.shape[0]
    y, saved = forward(p, x, mirror=mirror, keep=True)
    err = y - np.asarray(t, dtype=np.float64)
    L = float((err * err).sum() / (4.0 * n))
    layers = unpack(np.asarray(p, dtype=np.float64))
    grads = [None] * 4
    dz = q(err * (0.5 / n))                    # dL/dy
    for l in range(3, -1, -1):
        h, _ = saved[l]
        W, _ = layers[l]
        grads[l] = (h.T @ dz, dz.sum(axis=0))
        if l > 0:
            dh = dz @ q(W).T
            z_prev = saved[l - 1][1]
            dz = q(dh * gelu_d(z_prev))
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


class Adam:
    """Adam with bias correction, FP64 state."""

    def __init__(self, p, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.p = np.array(p, dtype=np.float64)
        self.m = np.zeros_like(self.p)
        self.v = np.zeros_like(self.p)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        self.p = self.p - self.lr * mh / (np.sqrt(vh) + self.eps)
        return self.p
