"""GPU parity of the compositional-initialization samplers (Sec. V) with the
oracle's definitions, and the sampling networks they compose into: the
conditional configuration sampler leaves grasps and placements as drawn,
composition picks satisfying actions, and the Sampling baseline's first
satisfying particle satisfies Eq. (3) by the oracle.

Bars: joint and grasp dimensions bit-exact (the uniform initializer's
draw); placement centres within 2e-6 m of the FP64 definition evaluated on
the same float32 yaw and Philox word (FP32 cos / sin and one FMA-free
interval map: a few float32 roundings at metre scale)."""
import numpy as np
import pytest

import oracle as O
from oracle.philox import uniform_init
from oracle.samplers import sampled_init
from paper_2411_11833_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("case,n", [("single", 1000), ("packing", 4099), ("six", 300)])
def test_seed_sampled_matches_oracle(case, n):
    from paper_2411_11833_amd.planner import GpuProblem
    prob = {"single": lambda: I.single_pick_place(0, 2), "packing": lambda: I.packing(0, 4),
            "six": lambda: I.packing(2, 3, n_objects=6, n_obstacles=4)}[case]()
    gp = GpuProblem(prob)
    X, M, V = gp.empty(n), gp.empty(n) + 3, gp.empty(n) + 4
    seed = 0xABCDEF0123
    gp.seed_sampled(seed, X, M, V, n)
    torch.cuda.synchronize()
    got = gp.to_rows(X, n).cpu().numpy()
    want = sampled_init(prob, n, seed)
    place = np.zeros(prob.dim, bool)
    for k in range(prob.skeleton.n_steps):
        place[I.STEP_DIM * k + 18:I.STEP_DIM * k + 20] = True
    lo, hi = prob.bounds()
    uni = uniform_init(lo, hi, n, seed)
    assert np.array_equal(got[:, ~place].view(np.uint32), uni[:, ~place].view(np.uint32))
    assert np.max(np.abs(got[:, place] - want[:, place])) <= 2e-6
    assert torch.all(M[:, :n] == 0) and torch.all(V[:, :n] == 0)
    # the containment term of every sampled placement is zero up to FP32 rounding
    T = O.terms(prob, got.astype(np.float64))
    for k in range(prob.skeleton.n_steps):
        assert np.all(T[:, I.TERMS_PER_STEP * k + I.TERM_NAMES.index("place")] <= 1e-6)


def test_configuration_sampler_keeps_grasps_and_placements():
    """The conditional sampler optimizes only the configurations: after its
    iterations every one-step particle keeps the grasp and placement the
    samplers drew, and the composition copies satisfying actions."""
    from paper_2411_11833_amd.sampling import CompositionalInit
    from paper_2411_11833_amd.planner import GpuProblem
    prob = I.packing(0, 6)
    gp = GpuProblem(prob)
    n_sub, n = 1024, 700
    ci = CompositionalInit(prob, n_sub)
    drawn = []
    ci.batch.seed(17, sampled=True)
    for k, g in enumerate(ci.batch.gps):
        drawn.append(g.to_rows(ci.batch.X[k], n_sub).cpu().numpy())
    X, M, V = gp.empty(n), gp.empty(n), gp.empty(n)
    ci.run(17, 300, X, M, V, n)
    torch.cuda.synchronize()
    comp = gp.to_rows(X, n).cpu().numpy()
    cnt = ci.count.cpu().numpy()
    for k, g in enumerate(ci.batch.gps):
        after = g.to_rows(ci.batch.X[k], n_sub).cpu().numpy()
        np.testing.assert_array_equal(after[:, 14:21], drawn[k][:, 14:21])
        assert not np.array_equal(after[:, :14], drawn[k][:, :14])
        blk = comp[:, I.STEP_DIM * k:I.STEP_DIM * (k + 1)]
        if cnt[k] > 0:
            idx = ci.idx[k, :cnt[k]].cpu().numpy()
            np.testing.assert_array_equal(blk, after[idx[np.arange(n) % cnt[k]]])
    print("satisfying actions per step after 300 configuration-sampler iterations:", cnt)
    ci.close()


def test_sampling_baseline_first_solution_satisfies_eq3():
    """The Sampling baseline on a single pick-place scene: fresh composed
    batches until one particle satisfies the whole skeleton; that particle
    passes the oracle's Eq. (3) (or lies within the mask band up to the term
    tolerance)."""
    from paper_2411_11833_amd.sampling import CompositionalInit, sampling_solve
    from paper_2411_11833_amd.planner import GpuProblem
    prob = I.single_pick_place(0, 0)
    gp = GpuProblem(prob)
    n = 1024
    ci = CompositionalInit(prob, n)
    r = sampling_solve(ci, gp, n, seed=3, ik_iters=2000, max_rounds=4)
    print("sampling baseline:", r.first_sat_iter, r.time_to_first_s, r.n_satisfied)
    assert r.first_sat_iter is not None
    X64 = r.solution.astype(np.float64)
    To = O.terms(prob, X64)
    eps = O.tolerance_vector(prob)
    nc = len(eps)
    assert np.all(To[:, :nc] <= eps + 1e-4 * np.abs(To[:, :nc]) + 2e-6)
    flip, _ = O.margins(prob, X64)
    outside = flip.min(1) > 1e-4
    assert np.all(O.mask(prob, To)[outside])
    ci.close()
