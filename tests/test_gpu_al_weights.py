"""GPU parity of the Lagrangian weight modes with the FP64 oracle, through
the C ABI: per-particle term weights in place of lambda (cost, gradient,
fused step, captured loop), the method-of-multipliers update and the PHR
augmented-Lagrangian weights.  Tolerances
as in the other parity tests: costs 1e-4 relative + 2e-6, gradients 1e-3
relative (kink margin >= 1e-5), one Adam update 1e-5 absolute; the
multiplier update is elementwise FP32 (one fused multiply-add, a max and an
add) against FP64 from the same FP32 inputs: 1e-6 relative + 1e-7.
"""
import numpy as np
import pytest

import oracle as O
from paper_2411_11833_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_parity import _adam, _close, _gp  # noqa: E402


def _cases():
    single = I.single_pick_place(0, 0)
    packing = I.packing(0, 0)
    selfc = I.packing(0, 0)
    selfc.skeleton.self_collision = 1
    motion = I.packing(robot_seed=1, scene_seed=2, n_objects=2, n_obstacles=2, waypoints=4)
    return {"single": single, "packing": packing, "self": selfc, "motion": motion}


def _weights(gp, prob, n, seed):
    """Random per-particle weights [n, n_terms] and the device table."""
    W = np.random.default_rng(seed).uniform(0.1, 5.0, (n, prob.n_terms)).astype(np.float32)
    Wd = gp.empty(n, rows=prob.n_terms)
    Wd[:, :n] = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
    return W, Wd


@pytest.mark.parametrize("case,n", [("single", 256), ("packing", 130), ("self", 96), ("motion", 40)])
def test_weighted_cost_and_gradient(case, n):
    prob = _cases()[case]
    gp = _gp(prob)
    X = I.uniform_particles(prob, n, seed=41)
    W, Wd = _weights(gp, prob, n, 42)
    gp.set_term_weights(Wd)
    Xd = gp.from_rows(X)
    c, T, m = gp.cost(Xd, n, terms=True)
    c2, G = gp.cost_grad(Xd, n)
    torch.cuda.synchronize()
    X64 = X.astype(np.float64)
    To = O.terms(prob, X64)
    Jo, Go = O.weighted_cost_and_grad(prob, X64, W.astype(np.float64))
    assert not _close(gp.to_rows(T, n).cpu().numpy(), To).any()          # terms stay unweighted
    assert not _close(c.cpu().numpy(), Jo).any()
    assert not _close(c2.cpu().numpy(), Jo).any()
    flip, kink = O.margins(prob, X64)
    outside = flip.min(1) > 1e-4
    assert np.array_equal(m.cpu().numpy()[outside].astype(bool), O.mask(prob, To)[outside])
    G = gp.to_rows(G, n).cpu().numpy().astype(np.float64)
    ok = kink >= 1e-5
    dn, gn = np.linalg.norm(G - Go, axis=1), np.linalg.norm(Go, axis=1)
    assert not (ok & (dn > 1e-3 * gn + 1e-5)).any()
    # back to lambda: the plain cost again
    gp.set_term_weights(None)
    c3, _, _ = gp.cost(Xd, n)
    torch.cuda.synchronize()
    assert not _close(c3.cpu().numpy(), To @ O.weights_vector(prob)).any()


def test_weighted_fused_step_and_captured_loop():
    prob = _cases()["packing"]
    n = 128
    gp = _gp(prob)
    X = I.uniform_particles(prob, n, seed=43)
    W, Wd = _weights(gp, prob, n, 44)
    gp.set_term_weights(Wd)
    Xd = gp.from_rows(X)
    Md, Vd = torch.zeros_like(Xd), torch.zeros_like(Xd)
    gp.step(Xd, Md, Vd, n, 1, _adam(n))
    torch.cuda.synchronize()
    X64 = X.astype(np.float64)
    _, Go = O.weighted_cost_and_grad(prob, X64, W.astype(np.float64))
    _, kink = O.margins(prob, X64)
    xo, _, _ = O.adam_step(X, np.zeros_like(X), np.zeros_like(X), Go, 1, grad_scale=1.0 / n)
    err = np.abs(gp.to_rows(Xd, n).cpu().numpy() - xo).max(1)
    assert np.all(err[kink >= 1e-5] <= 1e-5)
    # the captured loop reads the table at every launch: rewriting it in
    # place between replays is seen, and replays equal eager steps bit for bit
    outs = []
    for captured in (True, False):
        Xa, Ma, Va = gp.from_rows(X), torch.zeros_like(Xd), torch.zeros_like(Xd)
        Wd[:, :n] = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
        for r in range(2):
            if captured:
                gp.optimize(Xa, Ma, Va, n, 3 * r, 3, _adam(n))
            else:
                for t in range(3 * r + 1, 3 * r + 4):
                    gp.step(Xa, Ma, Va, n, t, _adam(n))
            Wd.mul_(1.5)
        torch.cuda.synchronize()
        outs.append(Xa.clone())
    assert torch.equal(outs[0], outs[1])
    gp.set_term_weights(None)


def test_al_update_matches_oracle():
    prob = _cases()["motion"]
    prob.skeleton.goal_cost = 1
    prob.skeleton.self_collision = 1
    n = 300
    gp = _gp(prob)
    X = I.uniform_particles(prob, n, seed=45)
    _, T, _ = gp.cost(gp.from_rows(X), n, terms=True)
    Th = gp.to_rows(T, n).cpu().numpy()
    Th[5, 3] = np.nan                                   # a non-finite term keeps its multiplier
    T[:, :n] = torch.from_numpy(np.ascontiguousarray(Th.T)).cuda()
    mu0 = np.random.default_rng(46).uniform(0, 2, Th.shape).astype(np.float32)
    mu = gp.empty(n, rows=prob.n_terms)
    mu[:, :n] = torch.from_numpy(np.ascontiguousarray(mu0.T)).cuda()
    W = gp.empty(n, rows=prob.n_terms)
    gp.al_update(T, n, 3.0, mu, W)
    torch.cuda.synchronize()
    muo, Wo = O.al_update(prob, Th.astype(np.float64), mu0.astype(np.float64), 3.0)
    mug, Wg = gp.to_rows(mu, n).cpu().numpy(), gp.to_rows(W, n).cpu().numpy()
    assert np.all(np.abs(mug - muo) <= 1e-6 * np.abs(muo) + 1e-7)
    assert np.all(np.abs(Wg - Wo) <= 1e-6 * np.abs(Wo) + 1e-7)
    assert mug[5, 3] == mu0[5, 3]
    assert np.any(mug == 0) and np.any(mug > mu0)


def test_phr_weights_match_oracle():
    """ct_al_weights against the oracle's PHR weights on the GPU's own FP32
    terms (both branches of the hinge, a NaN term, soft costs)."""
    prob = _cases()["motion"]
    prob.skeleton.goal_cost = 1
    n = 300
    gp = _gp(prob)
    X = I.uniform_particles(prob, n, seed=47)
    _, T, _ = gp.cost(gp.from_rows(X), n, terms=True)
    Th = gp.to_rows(T, n).cpu().numpy()
    Th[7, 2] = np.nan
    T[:, :n] = torch.from_numpy(np.ascontiguousarray(Th.T)).cuda()
    mu0 = np.random.default_rng(48).uniform(0, 2, Th.shape).astype(np.float32)
    mu = gp.empty(n, rows=prob.n_terms)
    mu[:, :n] = torch.from_numpy(np.ascontiguousarray(mu0.T)).cuda()
    W = gp.empty(n, rows=prob.n_terms)
    gp.al_weights(T, n, 3.0, mu, W)
    torch.cuda.synchronize()
    Wo = O.phr_weights(prob, Th.astype(np.float64), mu0.astype(np.float64), 3.0)
    Wg = gp.to_rows(W, n).cpu().numpy()
    assert np.all(np.abs(Wg - Wo) <= 1e-6 * np.abs(Wo) + 1e-7)
    assert np.array_equal(gp.to_rows(mu, n).cpu().numpy(), mu0)     # mu untouched
    lam = O.weights_vector(prob)
    nc = prob.n_constraint_terms
    assert np.any(Wg[:, :nc] == lam[None, :nc]) and np.any(Wg[:, :nc] > lam[None, :nc] + mu0[:, :nc])


def test_weights_with_another_ld_are_rejected():
    from paper_2411_11833_amd.binding import CtError
    prob = _cases()["single"]
    gp = _gp(prob)
    n = 100
    Wd = gp.empty(300, rows=prob.n_terms)     # ld 320, the particles' ld is 128
    gp.set_term_weights(Wd)
    with pytest.raises(CtError):
        gp.cost(gp.empty(n), n)
    gp.set_term_weights(None)


def test_al_solve_runs_and_reports_a_valid_solution():
    from paper_2411_11833_amd.planner import al_solve
    prob = _cases()["single"]
    gp = _gp(prob)
    for mode in ("phr", "dual"):
        r = al_solve(gp, 256, 3000, seed=7, rho=10.0, outer=50, mode=mode)
        print(f"al_solve single ({mode}):", r.first_sat_iter, r.n_satisfied)
        assert r.first_sat_iter is not None and r.n_satisfied >= 1


def test_al_weights_reach_a_satisfying_particle_sooner_than_fixed_weights():
    """What the multiplier updates gain over the fixed lambda of Eq. (2) on
    single pick-place (256 particles, same uniform seeds, same budget): a
    satisfying particle on every seed, and after fewer iterations than with
    fixed weights (or where fixed weights find none)."""
    from paper_2411_11833_amd.planner import al_solve, plain_solve
    prob = _cases()["single"]
    gp = _gp(prob)
    budget = 3000
    for seed in (4242, 4243, 4244):
        r_fixed = plain_solve(gp, 256, budget, seed=seed)
        for mode in ("phr", "dual"):
            r_al = al_solve(gp, 256, budget, seed=seed, rho=10.0, outer=50, mode=mode)
            print(f"seed {seed}: fixed lambda {r_fixed.first_sat_iter}, {mode} {r_al.first_sat_iter}")
            assert r_al.first_sat_iter is not None
            assert r_fixed.first_sat_iter is None or r_al.first_sat_iter < r_fixed.first_sat_iter


def test_many_skeleton_calls_use_lambda_even_with_weights_set():
    """A weight table set on a problem does not reach the many-skeleton
    launches (persistent or one launch per skeleton): results are bit-equal
    to the same batch without it."""
    from paper_2411_11833_amd.planner import GpuBatch
    robot = I.make_robot(0, n_spheres=60)
    probs = [I.random_skeleton_problem(s, robot) for s in (1, 2)]
    sizes = [131, 64]
    outs = []
    for weighted in (False, True):
        for persistent in (True, False):
            b = GpuBatch(probs, sizes)
            keep = []
            if weighted:
                for g, n in zip(b.gps, sizes):
                    W = g.empty(n, rows=g.n_terms).fill_(3.0)
                    keep.append(W)
                    g.set_term_weights(W)
            b.set_tuning(split=1, workgroups=0, persistent=persistent)
            b.seed(9)
            b.optimize(0, 6, _adam(1))
            torch.cuda.synchronize()
            outs.append([x.clone() for x in b.X])
            for g in b.gps:
                g.set_term_weights(None)
    for o in outs[1:]:
        for u, v in zip(outs[0], o):
            assert torch.equal(u, v)
