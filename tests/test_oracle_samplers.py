"""Pins of the oracle's compositional-initialization samplers (Sec. V) against
what their constraints fix: every placement keeps the object's footprint in
the goal region (corners rotated explicitly, not through the sampler's reach
formula) and the support is the whole feasible interval; every grasp
satisfies the Grasp constraint; the other dimensions are the uniform draws."""
import copy

import numpy as np

import oracle as O
from oracle.philox import uniform_init
from oracle.samplers import sampled_init
from paper_2411_11833_amd import inputs as I


def _corners(hx, hy, px, py, psi):
    c, s = np.cos(psi), np.sin(psi)
    out = []
    for sx in (-hx, hx):
        for sy in (-hy, hy):
            out.append((px + c * sx - s * sy, py + s * sx + c * sy))
    return np.array(out)   # [4, 2, n]


def test_placements_keep_the_footprint_in_the_region_and_span_it():
    prob = I.packing(0, 3)
    n = 20000
    X = sampled_init(prob, n, seed=99)
    rlo, rhi = prob.scene.region_lo, prob.scene.region_hi
    for k, obj in enumerate(prob.skeleton.object_of_step):
        o = I.STEP_DIM * k
        hx, hy = prob.scene.objects[obj, 4], prob.scene.objects[obj, 5]
        cr = _corners(hx, hy, X[:, o + 18], X[:, o + 19], X[:, o + 20])
        clear = np.minimum(cr - rlo[None, :, None], rhi[None, :, None] - cr)   # [4, 2, n]
        assert clear.min() >= -1e-12
        # tight: some footprint touches each side of the region within 1 mm
        for axis in (0, 1):
            assert (cr[:, axis] - rlo[axis]).min() < 1e-3
            assert (rhi[axis] - cr[:, axis]).min() < 1e-3
        # uniform along the feasible interval: the centre lies below the
        # middle of its interval about half of the time
        c, s = np.cos(X[:, o + 20]), np.sin(X[:, o + 20])
        ex = np.abs(cr[:, 0] - X[None, :, o + 18]).max(0)
        assert np.allclose(ex, np.abs(hx * c) + np.abs(hy * s))
        for axis in (0, 1):
            mid = 0.5 * (rlo[axis] + rhi[axis])
            assert abs((X[:, o + 18 + axis] < mid).mean() - 0.5) < 0.02
        # the two axes draw independent words
        assert abs(np.corrcoef(X[:, o + 18], X[:, o + 19])[0, 1]) < 0.05


def test_sampled_placements_zero_the_containment_term_and_grasps_the_grasp_term():
    prob = I.packing(0, 5)
    X = sampled_init(prob, 300, seed=7)
    T = O.terms(prob, X)
    for k in range(prob.skeleton.n_steps):
        tb = I.TERMS_PER_STEP * k
        assert np.all(T[:, tb + I.TERM_NAMES.index("place")] <= 1e-12)
        assert np.all(T[:, tb + I.TERM_NAMES.index("grasp")] == 0.0)


def test_other_dimensions_are_the_uniform_draws():
    prob = I.packing(1, 2, n_objects=3, n_obstacles=4)
    lo, hi = prob.bounds()
    X = sampled_init(prob, 500, seed=12345678901)
    U = uniform_init(lo, hi, 500, 12345678901).astype(np.float64)
    keep = np.ones(prob.dim, bool)
    for k in range(prob.skeleton.n_steps):
        keep[I.STEP_DIM * k + 18:I.STEP_DIM * k + 20] = False
    assert np.array_equal(X[:, keep], U[:, keep])
    assert not np.array_equal(X[:, ~keep], U[:, ~keep])


def test_region_narrower_than_the_footprint_takes_the_centre():
    prob = copy.deepcopy(I.single_pick_place(0, 1))
    sc = prob.scene
    sc.region_hi = sc.region_lo + np.array([0.01, 0.5])   # 1 cm wide: no object fits along x
    X = sampled_init(prob, 200, seed=3)
    assert np.allclose(X[:, 18], 0.5 * (sc.region_lo[0] + sc.region_hi[0]))
    assert np.ptp(X[:, 19]) > 0.1
