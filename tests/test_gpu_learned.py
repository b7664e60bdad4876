"""What the trained seed proposer gains over the method without it, on the
GPU: trained on converged particles of single pick-place training scenes,
its seeds let the plain optimizer reach a satisfying particle on held-out
scenes in fewer iterations (median over scenes) and at least as often as
from uniform seeds."""
import numpy as np
import pytest

from paper_2411_11833_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_learned_seeds_beat_uniform_on_held_out_scenes():
    from paper_2411_11833_amd import seeds as SD
    from paper_2411_11833_amd.planner import GpuProblem

    data = SD.collect(range(10000, 11024), n=1024, iters=3000, keep=64, make=SD.single_problem)
    assert len(data.targets) > 1000
    stats = SD.Stats.of(data)
    mlp = SD.GpuMlp(d_out=21, max_rows=1024 * 32)
    mlp.set_params(torch.from_numpy(I.mlp_init(mlp.dims, 0)))
    log = SD.train(mlp, data, stats, steps=5000, batch=1024, n_draws=32)
    assert log.losses[-1] < 0.9 * log.losses[0]
    prop = SD.Proposer(mlp, stats)

    n = 1024
    cost_u, cost_l, sat_u, sat_l = [], [], [], []
    for s in range(20000, 20006):
        prob = SD.single_problem(s)
        gp = GpuProblem(prob)
        X, M, V = gp.empty(n), gp.empty(n), gp.empty(n)
        gp.seed_uniform(11 + s, X, M, V, n)
        cost_u.append(float(gp.cost(X, n)[0].median().item()))
        prop.seed(prop.prepare(prob), 11 + s, X, M, V, n)
        cost_l.append(float(gp.cost(X, n)[0].median().item()))
        gp.close()
    cmp = SD.compare(prop, range(20000, 20006), n=256, budget=3000, make=SD.single_problem)
    sat_u = [r.first_sat_iter for r in cmp.uniform]
    sat_l = [r.first_sat_iter for r in cmp.learned]
    print("median seed cost uniform", np.round(cost_u, 3), "learned", np.round(cost_l, 3))
    print("first satisfying iteration uniform", sat_u, "learned", sat_l)
    budget = 3000
    assert sum(f is not None for f in sat_l) >= sum(f is not None for f in sat_u)
    assert np.median([f if f is not None else budget for f in sat_l]) < \
        np.median([f if f is not None else budget for f in sat_u])
    mlp.close()
