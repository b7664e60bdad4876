"""FP64 CPU oracle of the learned seed proposer -- TEST INFRASTRUCTURE ONLY.

Used by ``tests/`` (and nothing on the product path).  It shares no code with
the HIP kernels.

The paper initializes particles with samplers before optimizing them
(Sec. V "Particle Initialization"; learned generators are named there and in
the related work as one kind of sampler).  The proposer here is a multilayer
perceptron: the input row is the scene's features followed by Gaussian noise,
``depth`` hidden layers of width ``hidden`` with the exact (erf) GELU, and a
linear output layer giving one standardized particle.

Number format, written to be checked against the GPU kernels element by
element: BF16 round-to-nearest-even at the points where the GPU stores BF16
(the input row, every weight matrix, every hidden activation, and in the
backward pass every upstream gradient entering a product), everything else in
float64 here (FP32 with FP32 accumulation on the GPU).  ``bf16=False`` gives the
plain float64 network, the one the pins compare with library routines.

Training objective: implicit maximum likelihood estimation (Li and Malik,
"Implicit Maximum Likelihood Estimation", 2018): for every target row draw S
noise vectors, keep the draw whose output is nearest (squared Euclidean) to
the target, and take the mean squared error of that output.  Optional
per-entry weights W (0 or 1 in use: which target entries are trusted) enter
both the distance and the error.

Noise: Box and Muller's transform of uniforms from Philox4x32-10 (the same
counter-based generator as the uniform initializer).  Noise entry j of a row
with counter words (c0, c1) uses Philox(counter = (c0, c1, j // 4, 0), key =
(seed low, seed high)); words (w0, w1) give entries 4(j//4), 4(j//4)+1 and
(w2, w3) the next two, with u1 = 1 - (w >> 8) 2^-24 in (0, 1], u2 = (w >> 8)
2^-24, z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).

Parameter order (flat float32 on the GPU): for each layer W [out][in]
row-major, then b [out].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .philox import philox4x32_10

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


# --------------------------------------------------------------------------
# number format


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (8 exponent bits, 7 stored mantissa bits), to nearest
    with ties to even, after rounding to float32; returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, on: bool):
    return bf16_round(x) if on else np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# activation


def gelu(x):
    """x * Phi(x), Phi the standard normal CDF."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) * INV_SQRT_2PI


# --------------------------------------------------------------------------
# parameters


def layer_dims(d_in: int, hidden: int, depth: int, d_out: int) -> list[tuple[int, int]]:
    """[(in, out)] of the depth + 1 linear layers."""
    dims = [d_in] + [hidden] * depth + [d_out]
    return [(dims[i], dims[i + 1]) for i in range(depth + 1)]


def param_count(dims) -> int:
    return sum(i * o + o for i, o in dims)


def unflatten(params, dims) -> list[tuple[np.ndarray, np.ndarray]]:
    p = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for i, o in dims:
        W = p[off:off + i * o].reshape(o, i)
        off += i * o
        b = p[off:off + o]
        off += o
        out.append((W, b))
    assert off == p.size
    return out


def flatten(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


# --------------------------------------------------------------------------
# noise and input rows


def normal_noise(seed: int, c0, c1, d_noise: int) -> np.ndarray:
    """[rows, d_noise] standard normals for counter words c0[r], c1[r]."""
    c0 = np.asarray(c0, dtype=np.uint32).reshape(-1)
    c1 = np.asarray(c1, dtype=np.uint32).reshape(-1)
    rows, nb = c0.size, (d_noise + 3) // 4
    ctr = np.zeros((rows, nb, 4), dtype=np.uint32)
    ctr[..., 0] = c0[:, None]
    ctr[..., 1] = c1[:, None]
    ctr[..., 2] = np.arange(nb, dtype=np.uint32)[None, :]
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    w = philox4x32_10(ctr, key).astype(np.float64)
    u = np.floor(w / 256.0) * 2.0 ** -24          # (w >> 8) * 2^-24, in [0, 1)
    u1 = 1.0 - u[..., 0::2]                       # (0, 1]
    u2 = u[..., 1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty((rows, nb, 4))
    z[..., 0::2] = rad * np.cos(2.0 * math.pi * u2)
    z[..., 1::2] = rad * np.sin(2.0 * math.pi * u2)
    return z.reshape(rows, nb * 4)[:, :d_noise]


def input_rows(feats, feat_of_row, seed: int, c0, c1, d_noise: int) -> np.ndarray:
    """[rows, d_feat + d_noise]: the row's scene features, then its noise."""
    F = np.asarray(feats, dtype=np.float64)
    idx = np.asarray(feat_of_row, dtype=np.int64)
    return np.concatenate([F[idx], normal_noise(seed, c0, c1, d_noise)], axis=1)


# --------------------------------------------------------------------------
# network


def forward(layers, X, bf16: bool = True):
    """Y [rows, d_out] and the cache (layer inputs h, pre-activations z)."""
    h = _r(X, bf16)
    hs, zs = [h], []
    for li, (W, b) in enumerate(layers):
        z = h @ _r(W, bf16).T + b
        if li + 1 < len(layers):
            zs.append(z)
            h = _r(gelu(z), bf16)
            hs.append(h)
        else:
            return z, (hs, zs)


def backward(layers, cache, dY, bf16: bool = True) -> np.ndarray:
    """Flat gradient (parameter order) of sum(dY * Y) through the cached pass."""
    hs, zs = cache
    g = _r(dY, bf16)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (g.T @ hs[li], g.sum(0))
        if li:
            dh = g @ _r(W, bf16)
            g = _r(dh * gelu_grad(zs[li - 1]), bf16)
    return flatten(grads)


# --------------------------------------------------------------------------
# IMLE


def imle_select(Y, T, W=None) -> np.ndarray:
    """Y [B, S, d] outputs of S draws per target, T [B, d] targets, W [B, d]
    optional per-entry weights: index of the nearest draw (weighted squared
    Euclidean distance; the lowest index among equals)."""
    w = 1.0 if W is None else np.asarray(W, np.float64)[:, None, :]
    d2 = (w * (np.asarray(Y, np.float64) - np.asarray(T, np.float64)[:, None, :]) ** 2).sum(-1)
    return np.argmin(d2, axis=1)


def mse(Y, T, W=None):
    """sum of W (Y - T)^2 over rows and columns divided by their count
    (W = 1: the mean squared error), and its gradient w.r.t. Y."""
    Y, T = np.asarray(Y, np.float64), np.asarray(T, np.float64)
    w = 1.0 if W is None else np.asarray(W, np.float64)
    diff = Y - T
    n = diff.size
    return float((w * diff * diff).sum() / n), 2.0 * w * diff / n


def adam(p, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """Kingma-Ba update with bias correction (t is the 1-based step count)."""
    m1 = beta1 * m + (1 - beta1) * g
    v1 = beta2 * v + (1 - beta2) * g * g
    p1 = p - lr * (m1 / (1 - beta1 ** t)) / (np.sqrt(v1 / (1 - beta2 ** t)) + eps)
    return p1, m1, v1


def imle_step(params, m, v, t: int, dims, feats, feat_of_row, targets, n_draws: int, seed: int,
              d_noise: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, bf16: bool = True, weights=None):
    """One IMLE training step on B target rows (optional per-entry weights
    in the distance and the loss).

    Noise of draw s for target row b has counter words (b, s).  Returns
    (params, m, v, loss, chosen draw per row, gradient).
    """
    layers = unflatten(params, dims)
    T = np.asarray(targets, np.float64)
    B = T.shape[0]
    fr = np.asarray(feat_of_row)
    bb = np.repeat(np.arange(B), n_draws)
    ss = np.tile(np.arange(n_draws), B)
    Xall = input_rows(feats, fr[bb], seed, bb, ss, d_noise)
    Yall, _ = forward(layers, Xall, bf16)
    chosen = imle_select(Yall.reshape(B, n_draws, -1), T, weights)
    X = input_rows(feats, fr, seed, np.arange(B), chosen, d_noise)
    Y, cache = forward(layers, X, bf16)
    loss, dY = mse(Y, T, weights)
    g = backward(layers, cache, dY, bf16)
    p1, m1, v1 = adam(np.asarray(params, np.float64), m, v, g, t, lr, beta1, beta2, eps)
    return p1, m1, v1, loss, chosen, g


# --------------------------------------------------------------------------
# seeds


def destandardize(Y, mean, std, lo, hi, wrap) -> np.ndarray:
    """Particle rows from standardized outputs: y * std + mean, angles
    (wrap = 1) wrapped into [-pi, pi), then every coordinate clamped into
    [lo, hi] (the box the uniform initializer draws from)."""
    x = np.asarray(Y, np.float64) * np.asarray(std, np.float64) + np.asarray(mean, np.float64)
    w = np.asarray(wrap, bool)
    two_pi = 2.0 * math.pi
    xw = x - two_pi * np.floor((x + math.pi) / two_pi)
    x = np.where(w[None, :], xw, x)
    return np.clip(x, np.asarray(lo, np.float64), np.asarray(hi, np.float64))
