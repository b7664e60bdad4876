"""Compositional initialization (Sec. V "Particle Initialization") and the
Sampling baseline of Sec. VII.

The particles of a K-step pick-place skeleton are composed from the outputs
of parallel samplers, each solving a subgraph of the constraint network, as
the paper's sampling networks do:

  grasp sampler       grasps uniform in the valid grasp box (Grasp holds);
  placement sampler   placements whose footprint lies in the goal region
                      (StablePlace containment holds), ct_seed_sampled;
  configuration sampler, conditioned on both: the pick and place
                      configurations of one action, solved by the plain
                      optimizer on that action's cost with the grasp and the
                      placement frozen (the paper uses cuRobo's parallel IK;
                      here the same fused cost restricted to one action, i.e.
                      Kin at the pick and the place, joint limits, the
                      collision terms of the arm holding the object, and
                      the object at its placement, which no configuration
                      changes, so a colliding placement is rejected).

The K one-step problems (object k moved alone, the other objects where they
start) run together, one persistent many-skeleton launch per iteration.
Step k of composed particle i takes the i-th (cyclically) one-step particle
that satisfies every constraint of its action (Eq. 3), or, when none does,
one-step particle i as it stands: composition with rejection.  The paper's
method then refines the composed batch with the plain optimizer on the whole
skeleton, which resolves what no action saw alone (objects placed by earlier
steps, the goal cost); the Sampling baseline instead draws a fresh composed
batch, with no optimization of the whole skeleton, until one satisfies.

`conditional=False` keeps the earlier variant in which each one-step problem
optimizes its grasp-free dimensions jointly (placement included) from
uniform draws.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding as B
from . import inputs as I
from .planner import INT32_MAX, GpuBatch, GpuProblem, SolveResult, _stream, default_adam, grasp_frozen


def one_step_problems(prob: I.Problem) -> list[I.Problem]:
    """One problem per pick-place step: the same robot and scene, the
    skeleton reduced to that step's object."""
    return [I.Problem(prob.robot, prob.scene,
                      I.Skeleton(object_of_step=np.array([prob.skeleton.object_of_step[k]], dtype=np.int32)),
                      prob.weights, prob.tolerances)
            for k in range(prob.skeleton.n_steps)]


class CompositionalInit:
    """Buffers and handles for initializing one skeleton's particles by
    composition; reusable across calls (nothing is allocated per call)."""

    def __init__(self, prob: I.Problem, n_sub: int, device="cuda", conditional: bool = True):
        self.prob = prob
        self.n_sub = n_sub
        self.device = torch.device(device)
        self.conditional = conditional
        self.subs = one_step_problems(prob)
        self.batch = GpuBatch(self.subs, [n_sub] * len(self.subs), self.device, fixed_placements=conditional)
        K = len(self.subs)
        self.idx = torch.empty((K, n_sub), dtype=torch.int32, device=self.device)
        self.count = torch.empty(K, dtype=torch.int32, device=self.device)
        self.cost = torch.empty(n_sub, dtype=torch.float32, device=self.device)
        self.mask = torch.empty((K, n_sub), dtype=torch.uint8, device=self.device)

    def close(self):
        self.batch.close()
        for g in self.batch.gps:
            g.close()

    def run(self, seed: int, iters: int, X, M, V, n: int, chunk: int = 50):
        """Enqueue the samplers (grasps and placements drawn, then `iters`
        Adam steps of the configuration sampler; with conditional=False
        uniform draws and the joint one-step solve), the satisfaction masks of
        their particles, and the composition into X (M, V zeroed).  No host
        synchronization."""
        gb = self.batch
        gb.seed(seed, sampled=self.conditional)
        adam = default_adam(1)   # the batch uses 1/n per skeleton
        for t in range(0, iters, chunk):
            gb.optimize(t, min(chunk, iters - t), adam)
        self._compose(X, M, V, n)

    def _compose(self, X, M, V, n: int):
        """Masks of the one-step particles as they stand, then composition."""
        gb = self.batch
        st = _stream()
        for k, g in enumerate(gb.gps):
            B.ct_cost(g.handle, gb.X[k].data_ptr(), self.n_sub, gb.X[k].shape[1], self.cost.data_ptr(), None,
                      self.mask[k].data_ptr(), st)
            B.ct_compact(self.mask[k].data_ptr(), self.n_sub, self.idx[k].data_ptr(),
                         self.count[k:k + 1].data_ptr(), st)
            B.ct_gather_block(gb.X[k].data_ptr(), gb.X[k].shape[1], I.STEP_DIM, self.n_sub, self.idx[k].data_ptr(),
                              self.count[k:k + 1].data_ptr(), X.data_ptr(),
                              None if M is None else M.data_ptr(), None if V is None else V.data_ptr(),
                              X.shape[1], I.STEP_DIM * k, n, st)

    def seed_from(self, Xfull):
        """Seed the one-step problems from a whole-skeleton particle batch
        (e.g. a learned proposer's seeds): one-step problem k takes the rows
        of step k; moments zeroed."""
        gb = self.batch
        st = _stream()
        ld = Xfull.shape[1]
        for k in range(len(gb.gps)):
            B.ct_gather_block(Xfull.data_ptr() + 4 * I.STEP_DIM * k * ld, ld, I.STEP_DIM, ld, None, None,
                              gb.X[k].data_ptr(), gb.M[k].data_ptr(), gb.V[k].data_ptr(), gb.X[k].shape[1], 0,
                              self.n_sub, st)
        gb.first_sat.fill_(INT32_MAX)

    def solve(self, gp: GpuProblem, n: int, seed: int, max_iters: int = 2000, chunk: int = 100,
              first_check: int = 300, refine_budget: int = 2000, refine_chunk: int = 10,
              seeder=None) -> SolveResult:
        """Time to the first satisfying particle of the whole skeleton: the
        one-step problems run in chunks; after each chunk from `first_check`
        on, their satisfying particles are composed and the composed batch is
        tested (one cost launch; the host reads one flag).  When no composed
        particle satisfies by `max_iters`, the last composition is refined by
        the plain optimizer with stop at first.  `first_sat_iter` counts
        one-step iterations plus refinement iterations.  With `seeder(X, M,
        V)`, which fills a whole-skeleton batch of n_sub particles (timed),
        the one-step problems start from its step blocks instead of uniform
        draws."""
        gb = self.batch
        X, M, V = gp.empty(n), gp.empty(n), gp.empty(n)
        cost = torch.empty(n, dtype=torch.float32, device=gp.device)
        mask = torch.empty(n, dtype=torch.uint8, device=gp.device)
        Xs = gp.empty(self.n_sub) if seeder is not None else None
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        start = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        if seeder is None:
            gb.seed(seed, sampled=self.conditional)
        else:
            seeder(Xs, None, None)
            self.seed_from(Xs)
        adam1 = default_adam(1)
        done = 0
        while done < max_iters:
            c = min(chunk, max_iters - done)
            gb.optimize(done, c, adam1)
            done += c
            if done < first_check and done < max_iters:
                continue
            self._compose(X, M, V, n)
            B.ct_cost(gp.handle, X.data_ptr(), n, X.shape[1], cost.data_ptr(), None, mask.data_ptr(),
                      stream.cuda_stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            if bool(mask[:n].any().item()):
                wall = time.perf_counter() - t_wall
                sol = gp.to_rows(X, n)[mask[:n].bool()].cpu().numpy()
                return SolveResult(done, done, start.elapsed_time(ev) / 1e3, wall, int(mask[:n].sum().item()), sol)
        # refine the last composition
        adam = default_adam(n)
        frozen = grasp_frozen(gp.prob, gp.device)
        flag = torch.full((1,), INT32_MAX, dtype=torch.int32, device=gp.device)
        events = []
        t = 0
        while t < refine_budget:
            c = min(refine_chunk, refine_budget - t)
            gp.optimize(X, M, V, n, t, c, adam, frozen=frozen, cost=cost, mask=mask, first_sat=flag,
                        stop_at_first=True)
            t += c
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            events.append(e)
        torch.cuda.synchronize()
        f = int(flag.item())
        wall = time.perf_counter() - t_wall
        if f == INT32_MAX:
            return SolveResult(max_iters + refine_budget, None, None, wall, int(mask.sum().item()))
        ttf = start.elapsed_time(events[min(f // refine_chunk, len(events) - 1)]) / 1e3
        sol = gp.to_rows(X, n)[mask[:n].bool()].cpu().numpy()
        return SolveResult(max_iters + refine_budget, max_iters + f, ttf, wall, int(mask.sum().item()), sol)


def sampling_solve(ci: CompositionalInit, gp: GpuProblem, n: int, seed: int, ik_iters: int = 600,
                   max_rounds: int = 20, budget_s: float | None = None) -> SolveResult:
    """The Sampling baseline (Sec. VII): composed batches drawn again and
    again (fresh grasps and placements, `ik_iters` steps of the
    configuration sampler, composition), each checked against Eq. (3) on the
    whole skeleton, with no optimization of the composed particles.  Stops at
    the first satisfying particle, after `max_rounds` batches, or once the
    GPU time passes `budget_s`.  `first_sat_iter` counts configuration-sampler
    iterations over all rounds."""
    X, M, V = gp.empty(n), gp.empty(n), gp.empty(n)
    cost = torch.empty(n, dtype=torch.float32, device=gp.device)
    mask = torch.empty(n, dtype=torch.uint8, device=gp.device)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for r in range(max_rounds):
        ci.run(seed * 1000 + r, ik_iters, X, M, V, n)
        B.ct_cost(gp.handle, X.data_ptr(), n, X.shape[1], cost.data_ptr(), None, mask.data_ptr(), stream.cuda_stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        found = bool(mask[:n].any().item())
        t = start.elapsed_time(ev) / 1e3
        if found:
            sol = gp.to_rows(X, n)[mask[:n].bool()].cpu().numpy()
            return SolveResult((r + 1) * ik_iters, (r + 1) * ik_iters, t, time.perf_counter() - t_wall,
                               int(mask[:n].sum().item()), sol)
        if budget_s is not None and t > budget_s:
            break
    return SolveResult(max_rounds * ik_iters, None, None, time.perf_counter() - t_wall, 0)
