"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
published definition with numpy uint32 arithmetic -- TEST INFRASTRUCTURE
ONLY (the oracle side of the uniform initializer's bit-exact parity).

Round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products),
c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by the Weyl
constants (W0, W1) before every round after the first; ten rounds.
"""
import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)


def philox4x32_10(ctr, key):
    """ctr: uint32 [..., 4]; key: uint32 [..., 2] (broadcast).  Returns [..., 4]."""
    c = np.array(ctr, dtype=np.uint32, copy=True)
    k = np.array(key, dtype=np.uint32, copy=True)
    k0 = np.broadcast_to(k[..., 0], c.shape[:-1]).copy()
    k1 = np.broadcast_to(k[..., 1], c.shape[:-1]).copy()
    mask = np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = (k0 + W0).astype(np.uint32)
                k1 = (k1 + W1).astype(np.uint32)
            p0 = M0 * c[..., 0].astype(np.uint64)
            p1 = M1 * c[..., 2].astype(np.uint64)
            hi0, lo0 = (p0 >> np.uint64(32)).astype(np.uint32), (p0 & mask).astype(np.uint32)
            hi1, lo1 = (p1 >> np.uint64(32)).astype(np.uint32), (p1 & mask).astype(np.uint32)
            c = np.stack([hi1 ^ c[..., 1] ^ k0, lo1, hi0 ^ c[..., 3] ^ k1, lo0], -1)
    return c


def uniform_init(lo, hi, n: int, seed: int) -> np.ndarray:
    """The GPU uniform initializer's definition: dimension d of particle i
    takes word d % 4 of Philox(counter = (i, d // 4, 0, 0), key = (seed low
    32 bits, seed high 32 bits)), u = (w >> 8) * 2^-24, x = lo + (hi - lo) u
    evaluated in float32 (one rounding per operation).  Returns [n, dim]."""
    lo = np.asarray(lo, dtype=np.float32)
    hi = np.asarray(hi, dtype=np.float32)
    dim = lo.shape[0]
    nb = (dim + 3) // 4
    i = np.arange(n, dtype=np.uint32)[:, None]
    b = np.arange(nb, dtype=np.uint32)[None, :]
    ctr = np.zeros((n, nb, 4), dtype=np.uint32)
    ctr[..., 0] = i
    ctr[..., 1] = b
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    words = philox4x32_10(ctr, key).reshape(n, nb * 4)[:, :dim]
    u = (words >> np.uint32(8)).astype(np.float32) * np.float32(2.0 ** -24)
    width = (hi - lo).astype(np.float32)
    return (lo[None] + (width[None] * u).astype(np.float32)).astype(np.float32)
