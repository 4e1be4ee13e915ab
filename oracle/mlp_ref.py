"""FP64 reference of the Fourier-feature MLP surrogate -- TEST INFRASTRUCTURE ONLY.

Network (a learned stand-in for far-field winding-number queries; not part of
the paper, whose nearest item is its future-work remark about approximating
the fractional part of the formula):

    gamma(p) = [sin(2 pi G p), cos(2 pi G p)]            G: 32 x 3, fixed
    x1 = gelu(gamma W1 + b1)                             64 -> 128
    x2..x4 = gelu(x W + b)                               128 -> 128 (three layers)
    y = x4 W5 + b5                                       128 -> 1
    gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2
    loss = mean((y - t)^2);  Adam with bias correction.

Parameters are one flat vector in this order: W1 (64x128, row-major
[in][out]), b1, W2, b2, W3, b3, W4, b4, W5 (128), b5 -- 57,985 values.
`bf16=True` rounds the weights and the input of every layer to bfloat16
(round to nearest even), as the GPU kernels do before their matrix products.
`half=True` takes the inference kernel's operands instead: the bf16 weights of
the four hidden products carried into IEEE half precision (exact for |w| in
[2^-14, 65504]), the output layer's weights in bf16, and the input of every
layer rounded to half precision (round to nearest even).  GELU stays exact.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = [64, 128, 128, 128, 128, 1]
N_PARAMS = sum(SIZES[i] * SIZES[i + 1] + SIZES[i + 1] for i in range(5))


def offsets():
    off, o = [], 0
    for i in range(5):
        w = SIZES[i] * SIZES[i + 1]
        off.append((o, o + w, o + w + SIZES[i + 1]))
        o += w + SIZES[i + 1]
    return off


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    Ws, bs = [], []
    for i, (a, b, c) in enumerate(offsets()):
        Ws.append(theta[a:b].reshape(SIZES[i], SIZES[i + 1]))
        bs.append(theta[b:c])
    return Ws, bs


def round_bf16(a):
    """float -> bfloat16 (round to nearest, ties to even) -> float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def round_half(a):
    """float -> IEEE half (round to nearest even, saturated at 65504) -> float64."""
    return np.clip(np.asarray(a, np.float64), -65504.0, 65504.0).astype(np.float16).astype(np.float64)


def features(P, G):
    z = 2.0 * math.pi * (np.asarray(P, np.float64) @ np.asarray(G, np.float64).T)
    return np.concatenate([np.sin(z), np.cos(z)], axis=1)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, G, P, bf16=False, half=False):
    Ws, bs = unpack(theta)
    if half:
        r = round_half
        rw = [lambda a: round_half(round_bf16(a))] * 4 + [round_bf16]
    else:
        r = round_bf16 if bf16 else (lambda a: np.asarray(a, np.float64))
        rw = [r] * 5
    x = features(P, G)
    xs, zs = [], []
    for l in range(4):
        xi = r(x)
        xs.append(xi)
        z = xi @ rw[l](Ws[l]) + bs[l]
        zs.append(z)
        x = gelu(z)
    xi = r(x)
    xs.append(xi)
    y = xi @ rw[4](Ws[4])[:, 0] + bs[4][0]
    return y, (xs, zs)


def loss_and_grad(theta, G, P, t, bf16=False):
    """MSE loss and its gradient with respect to the flat parameter vector."""
    Ws, bs = unpack(theta)
    r = round_bf16 if bf16 else (lambda a: np.asarray(a, np.float64))
    y, (xs, zs) = forward(theta, G, P, bf16)
    n = len(y)
    d = y - np.asarray(t, np.float64)
    loss = float(np.mean(d * d))
    dy = 2.0 * d / n
    gW = [None] * 5
    gb = [None] * 5
    gW[4] = (xs[4].T @ dy)[:, None]
    gb[4] = np.array([dy.sum()])
    dx = np.outer(dy, r(Ws[4])[:, 0])
    for l in range(3, -1, -1):
        dz = dx * gelu_grad(zs[l])
        gW[l] = xs[l].T @ dz
        gb[l] = dz.sum(axis=0)
        if l > 0:
            dx = dz @ r(Ws[l]).T
    g = np.concatenate([np.concatenate([gW[i].ravel(), gb[i]]) for i in range(5)])
    return loss, g


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
