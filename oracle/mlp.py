"""FP64 reference of the surrogate MLP -- TEST INFRASTRUCTURE ONLY.

The paper picks designs with a global optimizer (efficient global optimization with a Gaussian-
process surrogate, Sec. II.A).  The learned screen here is a multilayer perceptron
12 -> 256 -> 256 -> 256 -> 256 -> 3 with exact-erf GELU between layers, whose outputs are the
z-scored switching field, the z-scored log switching time and the logit of the switching
probability of a design.

Precision model of the GPU kernels, reproduced here in FP64 arithmetic: every operand of a
matrix product (weights, layer inputs, output gradients) is rounded to bfloat16 (round to
nearest even); products are accumulated exactly-ish (FP64 here, FP32 on the GPU); bias, GELU,
loss and Adam work on full-precision values.

Loss (per batch of B samples, mask m_b = 1 where the design switched):
  L = (1/B) sum_b [ m_b ((y0 - t0)^2 + (y1 - t1)^2) + softplus(y2) - t2 y2 ]
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = (12, 256, 256, 256, 256, 3)


def bf16_round(x) -> np.ndarray:
    """float -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def param_count(sizes=SIZES) -> int:
    return sum(sizes[i] * sizes[i + 1] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(theta, sizes=SIZES):
    """Flat parameter vector -> [(W [out][in], b [out])] in layer order."""
    out, o = [], 0
    for i in range(len(sizes) - 1):
        ni, no = sizes[i], sizes[i + 1]
        W = theta[o:o + ni * no].reshape(no, ni); o += ni * no
        b = theta[o:o + no]; o += no
        out.append((W, b))
    return out


def _identity(x):
    return np.asarray(x, dtype=np.float64)


def forward(theta, X, sizes=SIZES, rounding=True):
    """Returns (Y [B][3], cache).  rounding=False evaluates the exact FP64 network."""
    rd = bf16_round if rounding else _identity
    layers = unpack(np.asarray(theta, dtype=np.float64), sizes)
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = rd(a) @ rd(W).T + b
        cache.append((a, z))
        a = gelu(z) if li < len(layers) - 1 else z
    return a, cache


def loss_and_dy(Y, T, mask):
    B = Y.shape[0]
    m = np.asarray(mask, dtype=np.float64)
    d0, d1 = Y[:, 0] - T[:, 0], Y[:, 1] - T[:, 1]
    z, t = Y[:, 2], T[:, 2]
    sp = np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z)))
    L = (m * (d0 * d0 + d1 * d1) + sp - t * z).sum() / B
    dY = np.empty_like(Y)
    dY[:, 0] = 2.0 * m * d0 / B
    dY[:, 1] = 2.0 * m * d1 / B
    dY[:, 2] = (1.0 / (1.0 + np.exp(-z)) - t) / B
    return L, dY


def backward(theta, cache, dY, sizes=SIZES, rounding=True):
    """Gradient of the loss w.r.t. the flat parameter vector."""
    rd = bf16_round if rounding else _identity
    layers = unpack(np.asarray(theta, dtype=np.float64), sizes)
    grads = [None] * len(layers)
    g = dY
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        a, z = cache[li]
        dz = g if li == len(layers) - 1 else g * gelu_grad(z)
        dW = rd(dz).T @ rd(a)
        db = dz.sum(0)
        grads[li] = (dW, db)
        if li > 0:
            g = rd(dz) @ rd(W)
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def loss_grad(theta, X, T, mask, sizes=SIZES, rounding=True):
    Y, cache = forward(theta, X, sizes, rounding)
    L, dY = loss_and_dy(Y, T, mask)
    return L, backward(theta, cache, dY, sizes, rounding)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int, sizes=SIZES) -> np.ndarray:
    """He-uniform weights, zero biases (the seeded draw is an input to both sides)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        ni, no = sizes[i], sizes[i + 1]
        lim = math.sqrt(6.0 / ni)
        parts.append(rng.uniform(-lim, lim, size=no * ni))
        parts.append(np.zeros(no))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def topk_reference(score, k):
    """Indices of the k largest scores, ties to the lower index, ordered by (score desc, index)."""
    s = np.asarray(score, dtype=np.float32)
    order = np.lexsort((np.arange(s.size), -s.astype(np.float64)))
    return order[:k]
