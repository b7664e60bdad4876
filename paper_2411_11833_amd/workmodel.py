"""Algorithmic work per particle-iteration (cost + gradient + Adam), used to
place measured kernel times on the roofline.

Per-operation model (FMA = 2 flops, other arithmetic = 1; transcendental
sin / cos / sqrt / rsq / atan2 counted apart and not as flops):
  * one sphere-vs-box pair: 27 flops forward (offset, rotate into the box
    frame, |p| - h, clamp, squared norm, hinge) + 25 flops adjoint
    (d pen / d centre, rotation back, accumulation) -- the dense count a
    tape-based autodiff of the same cost would spend on every pair;
  * forward kinematics: 90 flops per joint and configuration;
  * one sphere transform to world: 18 flops;
  * Adam: 15 flops per coordinate;
  * one robot self-collision sphere pair (with the constraint on): 11 flops
    forward (difference, squared norm, radius sum, hinge) + 8 adjoint.
HBM bytes: X, M and V read and written once per coordinate (24 B) plus the
per-particle cost (4 B) and mask (1 B).
"""
from __future__ import annotations

from dataclasses import dataclass

from . import inputs as I

PAIR_FWD, PAIR_BWD = 27, 25
FK_PER_JOINT = 90
SPHERE_TF = 18
ADAM_PER_COORD = 15
SELF_FWD, SELF_BWD = 11, 8


def self_pair_count(sphere_link) -> int:
    """Robot sphere pairs on links two or more apart (per configuration)."""
    n = [0] * 10
    for L in sphere_link:
        n[int(L)] += 1
    return sum(n[a] * n[b] for a in range(10) for b in range(a + 2, 10))


@dataclass
class Work:
    pairs: int
    sphere_instances: int
    configs: int
    flops: int
    bytes: int


def per_particle_iteration(prob: I.Problem) -> Work:
    K = prob.skeleton.n_steps
    sc = prob.scene
    n_rs = prob.robot.spheres.shape[0]
    n_os = sc.obj_spheres.shape[1]
    n_boxes = 1 + len(sc.obstacles) + (len(sc.objects) - K) + (K - 1)   # boxes of one step
    configs = 2 * K
    spheres_per_config = n_rs + n_os           # robot + held object
    inst = configs * spheres_per_config + K * n_os   # + each placed object
    W = prob.skeleton.waypoints
    if W > 0:
        wp_configs = 2 * K * W
        configs += wp_configs
        inst += wp_configs * n_rs + K * W * n_os     # holding transitions carry the object
    pairs = inst * n_boxes
    flops = (pairs * (PAIR_FWD + PAIR_BWD) + configs * 7 * FK_PER_JOINT + inst * SPHERE_TF
             + prob.dim * ADAM_PER_COORD)
    if prob.skeleton.self_collision:
        flops += 2 * K * self_pair_count(prob.robot.sphere_link) * (SELF_FWD + SELF_BWD)
    nbytes = 24 * prob.dim + 5
    return Work(pairs=pairs, sphere_instances=inst, configs=configs, flops=flops, bytes=nbytes)


def method_flops(w: Work, penetrating_pairs: float) -> float:
    """Flops the method itself needs per particle-iteration: every pair's
    forward test, the adjoint only of the pairs that penetrate (the hinge
    has zero derivative elsewhere), and the rest of the dense model."""
    return w.flops - w.pairs * PAIR_BWD + penetrating_pairs * PAIR_BWD
