"""Samplers of compositional particle initialization -- TEST INFRASTRUCTURE
ONLY (the oracle side of the GPU samplers' parity; the product path never
imports it).

Sec. V composes parallel samplers, each solving a subgraph of the constraint
network: a grasp sampler for the Grasp constraint, a placement sampler for
the stable placement, and a configuration sampler conditioned on both (the
paper's cuRobo IK; here the same fused cost, optimized over the
configurations only).  The first two are fixed here by their definitions:

  grasp       (gx, gy, gz) uniform in the valid grasp box, yaw uniform in
              [-pi, pi): every draw satisfies the Grasp constraint;
  placement   yaw psi uniform in [-pi, pi); the footprint (half extents
              hx, hy) turned by psi reaches e_x = |hx cos psi| + |hy sin psi|
              and e_y = |hx sin psi| + |hy cos psi| from its centre, so the
              centre is drawn uniformly in [lo + e, hi - e] on each axis of
              the goal region: every corner lies in the region, i.e. the
              containment term of StablePlace is zero.  When the region is
              narrower than 2 e on an axis no centre keeps the footprint in,
              and the centre of the region is taken.
  configurations (the starting points of the conditional configuration
              sampler) uniform in the joint limits.

Random numbers: the same Philox4x32-10 words as the uniform initializer
(dimension d of particle i takes word d % 4 of the block (i, d // 4)), so
every dimension but the placement centre equals the uniform draw and the
centre uses its own dimension's word u, mapped to [lo + e, hi - e].
Arithmetic in float64 from the float32 values of u and psi.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10, uniform_init

STEP_DIM = 21


def _words_u(n: int, dim: int, seed: int) -> np.ndarray:
    """u = (w >> 8) 2^-24 of every (particle, dimension), as float64 (exact)."""
    nb = (dim + 3) // 4
    ctr = np.zeros((n, nb, 4), dtype=np.uint32)
    ctr[..., 0] = np.arange(n, dtype=np.uint32)[:, None]
    ctr[..., 1] = np.arange(nb, dtype=np.uint32)[None, :]
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    w = philox4x32_10(ctr, key).reshape(n, nb * 4)[:, :dim]
    return (w >> np.uint32(8)).astype(np.float64) * 2.0 ** -24


def footprint_reach(hx: float, hy: float, psi):
    """Half extents along world x and y of an hx x hy footprint turned by psi."""
    c, s = np.cos(psi), np.sin(psi)
    return np.abs(hx * c) + np.abs(hy * s), np.abs(hx * s) + np.abs(hy * c)


def sampled_init(prob, n: int, seed: int) -> np.ndarray:
    """[n, dim] float64 particles from the grasp, placement and configuration
    samplers (definitions in the module docstring)."""
    lo, hi = prob.bounds()
    X = uniform_init(lo, hi, n, seed).astype(np.float64)
    U = _words_u(n, prob.dim, seed)
    rlo, rhi = prob.scene.region_lo, prob.scene.region_hi
    for k, obj in enumerate(prob.skeleton.object_of_step):
        o = STEP_DIM * k
        hx, hy = prob.scene.objects[obj, 4], prob.scene.objects[obj, 5]
        ex, ey = footprint_reach(hx, hy, X[:, o + 20])
        for axis, e in ((0, ex), (1, ey)):
            a, b = rlo[axis] + e, rhi[axis] - e
            X[:, o + 18 + axis] = np.where(b >= a, a + (b - a) * U[:, o + 18 + axis], 0.5 * (rlo[axis] + rhi[axis]))
    return X
