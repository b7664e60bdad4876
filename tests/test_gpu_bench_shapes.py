"""Oracle parity at the launch shapes the benchmark times.

The benchmark runs the fused step at 8192 particles (four-object packing,
84-D, the split its autotuner picks, grasps frozen), the waypoint motion cost
at 16384 particles (136 configurations per particle, eight obstacles), five-
and six-step skeletons, and the persistent many-skeleton kernel.  Each case
here launches the GPU at that shape and checks against the FP64 oracle either
every particle (when the oracle finishes in seconds) or a sample of
particles that includes the first and the last workgroup.

Bars (Eqs. 2-4 and the Adam step of Sec. IV-B):
  terms, costs     |d| <= 1e-4 |oracle| + 2e-6
  gradients        per particle with kink margin >= 1e-5:
                   ||d g|| <= 1e-3 ||g|| + 1e-5; element-wise 1e-3 relative on
                   elements >= 1% of max |g|
  one Adam update  |d x'| <= 1e-5 absolute (kink margin >= 1e-5)
  masks            bit-exact for particles outside the 1e-4 flip-margin band
"""
import numpy as np
import pytest

import oracle as O
from paper_2411_11833_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

INT32_MAX = 2 ** 31 - 1


def _close(got, want, rtol=1e-4, atol=2e-6):
    return np.abs(np.asarray(got, np.float64) - want) > rtol * np.abs(want) + atol


def _sample(n, k=40, tail=16):
    """k particles spread over the batch plus the last `tail` (the last
    workgroup, which may be partly empty)."""
    return np.unique(np.concatenate([np.linspace(0, n - 1, k).astype(int), np.arange(max(0, n - tail), n)]))


def _grad_ok(G, Go, ok):
    dn = np.linalg.norm(G - Go, axis=1)
    gn = np.linalg.norm(Go, axis=1)
    bad = ok & (dn > 1e-3 * gn + 1e-5)
    assert not bad.any(), f"gradient norm error at {np.flatnonzero(bad)[:5]}: {dn[bad][:5]} vs {gn[bad][:5]}"
    big = np.abs(Go) >= 0.01 * np.abs(Go).max(1, keepdims=True)
    rel = np.abs(G - Go) / np.maximum(np.abs(Go), 1e-30)
    bad_e = ok[:, None] & big & (rel > 1e-3)
    assert not bad_e.any(), f"gradient element error at {np.argwhere(bad_e)[:5]}"


def _check_sampled(prob, gp, X, n, idx):
    """Terms, cost, mask and gradient of a GPU batch of n particles (device
    SoA X) against the oracle on the rows idx."""
    c, T, m = gp.cost(X, n, terms=True)
    _, G = gp.cost_grad(X, n)
    torch.cuda.synchronize()
    rows = gp.to_rows(X, n).cpu().numpy()[idx].astype(np.float64)
    To = O.terms(prob, rows)
    Tg = gp.to_rows(T, n).cpu().numpy()[idx]
    bad = _close(Tg, To)
    assert not bad.any(), f"terms differ at {np.argwhere(bad)[:5]}: {Tg[bad][:5]} vs {To[bad][:5]}"
    Jo, Go = O.cost_and_grad(prob, rows)
    assert not _close(c.cpu().numpy()[idx], Jo).any()
    flip, kink = O.margins(prob, rows)
    outside = flip.min(1) > 1e-4
    assert np.array_equal(m.cpu().numpy()[idx][outside].astype(bool), O.mask(prob, To)[outside])
    ok = kink >= 1e-5
    _grad_ok(gp.to_rows(G, n).cpu().numpy()[idx].astype(np.float64), Go, ok)
    print(f"n={n}: {len(idx)} sampled, {int(ok.sum())} kink-safe, {int(outside.sum())} outside the mask band")
    assert ok.mean() >= 0.75 and outside.mean() >= 0.75


# ----------------------------------------------------------------------------- motion


def _motion_bench():
    # the benchmark's motion workload: packing scene 0 (4 objects, 8 obstacles),
    # 16 interior waypoints per transition
    return I.packing(robot_seed=0, scene_seed=0, waypoints=16)


@pytest.mark.parametrize("split,n", [(1, 1024), (2, 1000)])
def test_motion_bench_scene(split, n):
    from paper_2411_11833_amd.planner import GpuProblem
    prob = _motion_bench()
    gp = GpuProblem(prob)
    gp.set_split(split)
    X = gp.empty(n)
    gp.seed_uniform(31, X, None, None, n)
    _check_sampled(prob, gp, X, n, _sample(n, k=32, tail=16))


def test_motion_bench_full_size():
    """16384 particles, the split the benchmark's autotuner picks."""
    from paper_2411_11833_amd.planner import GpuProblem
    prob = _motion_bench()
    gp = GpuProblem(prob)
    n = 16384
    X = gp.empty(n)
    gp.seed_uniform(31, X, None, None, n)
    split = gp.autotune(X, n)
    print("autotuned split", split)
    _check_sampled(prob, gp, X, n, _sample(n, k=24, tail=12))


def test_motion_bench_fused_step():
    """One fused motion step (cost, recomputing adjoint, Adam) at 16384
    particles against the oracle's Adam step on a sample."""
    from paper_2411_11833_amd.planner import GpuProblem, default_adam, grasp_frozen
    prob = _motion_bench()
    gp = GpuProblem(prob)
    n = 16384
    X = gp.empty(n)
    gp.seed_uniform(32, X, None, None, n)
    gp.autotune(X, n)
    _fused_step_sampled(prob, gp, X, n, grasp_frozen(prob), default_adam(n), _sample(n, k=24, tail=12))


# ----------------------------------------------------------------------------- fused step at full size


def _fused_step_sampled(prob, gp, X, n, frozen, adam, idx, warm=10):
    """`warm` eager steps (so M and V are not zero), then one more step with
    cost and mask; compare that step's update with the oracle's Adam step
    from the oracle gradient on the sampled rows."""
    M, V = gp.empty(n), gp.empty(n)
    for t in range(1, warm + 1):
        gp.step(X, M, V, n, t, adam, frozen=frozen)
    torch.cuda.synchronize()
    x0, m0, v0 = (gp.to_rows(a, n).cpu().numpy()[idx] for a in (X, M, V))
    cost = torch.empty(n, device="cuda")
    mask = torch.empty(n, dtype=torch.uint8, device="cuda")
    gp.step(X, M, V, n, warm + 1, adam, frozen=frozen, cost=cost, mask=mask)
    torch.cuda.synchronize()
    x64 = x0.astype(np.float64)
    Jo, Go = O.cost_and_grad(prob, x64)
    assert not _close(cost.cpu().numpy()[idx], Jo).any()
    flip, kink = O.margins(prob, x64)
    ok = kink >= 1e-5
    fz = frozen.cpu().numpy() if frozen is not None else None
    xo, mo, vo = O.adam_step(x0, m0, v0, Go, warm + 1, lr=adam.lr, grad_scale=adam.grad_scale, frozen=fz)
    xg = gp.to_rows(X, n).cpu().numpy()[idx]
    err = np.abs(xg - xo).max(1)
    assert np.all(err[ok] <= 1e-5), (err[ok].max(), np.flatnonzero(err > 1e-5)[:5])
    if fz is not None:
        assert np.array_equal(xg[:, fz.astype(bool)], x0[:, fz.astype(bool)])
    outside = flip.min(1) > 1e-4
    To = O.terms(prob, x64)
    assert np.array_equal(mask.cpu().numpy()[idx][outside].astype(bool), O.mask(prob, To)[outside])
    print(f"fused step n={n}: {len(idx)} sampled, {int(ok.sum())} kink-safe, max |dx'| {err[ok].max():.2e}")
    assert ok.mean() >= 0.75


@pytest.mark.parametrize("split", [1, 2, 4])
@pytest.mark.parametrize("fixed_grasps", [True, False])
def test_packing_fused_step_full_size(split, fixed_grasps):
    """The benchmark's headline launch: 8192 packing particles, one fused
    step; splits 1, 2 and 4, grasps frozen (the benchmark) and free."""
    from paper_2411_11833_amd.planner import GpuProblem, default_adam, grasp_frozen
    prob = I.packing(0, 0)
    gp = GpuProblem(prob)
    gp.set_split(split)
    n = 8192
    X = gp.empty(n)
    gp.seed_uniform(7, X, None, None, n)
    fz = grasp_frozen(prob) if fixed_grasps else None
    _fused_step_sampled(prob, gp, X, n, fz, default_adam(n), _sample(n))


# ----------------------------------------------------------------------------- five steps


def _five_steps():
    return I.packing(robot_seed=3, scene_seed=4, n_objects=5, n_obstacles=4)


@pytest.mark.parametrize("split", [1, 2, 4])
def test_five_step_skeleton(split):
    """K = 5 through the per-skeleton kernels: every particle of a ragged
    batch, terms, cost, mask and gradient."""
    from paper_2411_11833_amd.planner import GpuProblem
    prob = _five_steps()
    assert prob.skeleton.n_steps == 5
    gp = GpuProblem(prob)
    gp.set_split(split)
    n = 53
    X = gp.from_rows(I.uniform_particles(prob, n, seed=51))
    _check_sampled(prob, gp, X, n, np.arange(n))


def test_five_step_fused_step():
    from paper_2411_11833_amd.planner import GpuProblem, default_adam, grasp_frozen
    prob = _five_steps()
    gp = GpuProblem(prob)
    n = 3000
    X = gp.empty(n)
    gp.seed_uniform(52, X, None, None, n)
    _fused_step_sampled(prob, gp, X, n, grasp_frozen(prob), default_adam(n), _sample(n, k=32, tail=16))


# ----------------------------------------------------------------------------- persistent batch kernel


@pytest.mark.parametrize("split", [1, 2])
def test_batch_kernel_against_oracle(split):
    """The persistent many-skeleton kernel against the oracle directly (not
    only against per-skeleton launches): skeletons of every length K = 1..6,
    one step from uniform seeds, then a second step from non-zero moments;
    per skeleton its cost and mask (before the update) and its update are
    compared on a sample including the last tile."""
    from paper_2411_11833_amd.planner import GpuBatch, default_adam
    robot = I.make_robot(0, n_spheres=60)
    seeds = (1, 2, 3, 4, 6, 9)   # K = 3 4 2 5 1 6
    probs = [I.random_skeleton_problem(s, robot) for s in seeds]
    assert sorted(p.skeleton.n_steps for p in probs) == [1, 2, 3, 4, 5, 6]
    sizes = [131, 64, 200, 77, 256, 45]
    b = GpuBatch(probs, sizes)
    b.set_tuning(split=split, workgroups=37)
    b.seed(11)
    adam = default_adam(1)   # the batch applies 1/N_b per skeleton itself
    b.step(1, adam)
    torch.cuda.synchronize()
    # second step, recording per skeleton what went in
    before = []
    for s, (prob, n) in enumerate(zip(probs, sizes)):
        g = b.gps[s]
        before.append(tuple(g.to_rows(a, n).cpu().numpy() for a in (b.X[s], b.M[s], b.V[s])))
    b.step(2, adam)
    torch.cuda.synchronize()
    for s, (prob, n) in enumerate(zip(probs, sizes)):
        g = b.gps[s]
        idx = _sample(n, k=24, tail=8)
        x0, m0, v0 = (a[idx] for a in before[s])
        x64 = x0.astype(np.float64)
        Jo, Go = O.cost_and_grad(prob, x64)
        assert not _close(b.cost[s].cpu().numpy()[idx], Jo).any(), s
        flip, kink = O.margins(prob, x64)
        To = O.terms(prob, x64)
        outside = flip.min(1) > 1e-4
        assert np.array_equal(b.mask[s].cpu().numpy()[idx][outside].astype(bool), O.mask(prob, To)[outside]), s
        fz = b.frozen[s].cpu().numpy() if b.frozen[s] is not None else None
        xo, _, _ = O.adam_step(x0, m0, v0, Go, 2, lr=adam.lr, grad_scale=1.0 / n, frozen=fz)
        xg = g.to_rows(b.X[s], n).cpu().numpy()[idx]
        ok = kink >= 1e-5
        err = np.abs(xg - xo).max(1)
        assert np.all(err[ok] <= 1e-5), (s, err[ok].max())
        print(f"skeleton {s} (K={prob.skeleton.n_steps}, n={n}): {len(idx)} sampled, {int(ok.sum())} kink-safe, "
              f"max |dx'| {err[ok].max():.2e}")
        assert ok.mean() >= 0.75
