"""Torch-facing wrapper over the C ABI: PyTorch supplies device memory and
the stream; every step of the particle path runs in the HIP library.

* ``GpuProblem`` owns a problem handle and allocates particle buffers in the
  library's dimension-major layout (``[dim, ld]``, ld a multiple of 64).
* ``plain_solve`` is the paper's Optimization baseline (Sec. VII): uniform
  initialization within bounds, then Adam on the batch-mean cost of Eq. (4),
  stopping at the first satisfying particle (Sec. IV-B) or at the budget.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

import torch

from . import binding as B
from . import inputs as I


def padded(n: int) -> int:
    return max(64, ((n + 63) // 64) * 64)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class GpuProblem:
    """A created problem handle plus buffer helpers."""

    def __init__(self, prob: I.Problem, device: str | torch.device = "cuda"):
        self.prob = prob
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.handle = B.ct_problem_create(prob)
        self.dim, self.n_terms, self.n_constraint = B.ct_problem_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            B.ct_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- buffers
    def empty(self, n: int, rows: int | None = None) -> torch.Tensor:
        return torch.zeros((rows or self.dim, padded(n)), dtype=torch.float32, device=self.device)

    def from_rows(self, x_rows) -> torch.Tensor:
        """[n, dim] host/device rows -> [dim, ld] device SoA buffer."""
        x = torch.as_tensor(x_rows, dtype=torch.float32)
        out = self.empty(x.shape[0])
        out[:, : x.shape[0]] = x.T.to(self.device)
        return out

    @staticmethod
    def to_rows(buf: torch.Tensor, n: int) -> torch.Tensor:
        return buf[:, :n].T.contiguous()

    # ---- calls (argument marshalling only)
    def seed_uniform(self, seed: int, X, M=None, V=None, n: int | None = None):
        n = X.shape[1] if n is None else n
        B.ct_seed_uniform(self.handle, seed, X.data_ptr(), M.data_ptr() if M is not None else None,
                          V.data_ptr() if V is not None else None, n, X.shape[1], _stream())

    def seed_sampled(self, seed: int, X, M=None, V=None, n: int | None = None):
        """The grasp, placement and configuration samplers (ct_seed_sampled)."""
        n = X.shape[1] if n is None else n
        B.ct_seed_sampled(self.handle, seed, X.data_ptr(), M.data_ptr() if M is not None else None,
                          V.data_ptr() if V is not None else None, n, X.shape[1], _stream())

    def cost(self, X, n: int, terms: bool = False, mask: bool = True):
        c = torch.empty(n, dtype=torch.float32, device=self.device)
        T = self.empty(n, rows=self.n_terms) if terms else None
        m = torch.empty(n, dtype=torch.uint8, device=self.device) if mask else None
        B.ct_cost(self.handle, X.data_ptr(), n, X.shape[1], c.data_ptr(), T.data_ptr() if T is not None else None,
                  m.data_ptr() if m is not None else None, _stream())
        return c, T, m

    def feasibility(self, terms, n: int, penalty: float | None = None):
        """Eq. (5) on a terms buffer from cost(..., terms=True): per-constraint
        satisfying counts (int32 [n_constraint]) and H (float [1]), on the
        device; the penalty defaults to -n."""
        counts = torch.empty(self.n_constraint, dtype=torch.int32, device=self.device)
        H = torch.empty(1, dtype=torch.float32, device=self.device)
        B.ct_feasibility(self.handle, terms.data_ptr(), n, terms.shape[1], float(-n if penalty is None else penalty),
                         counts.data_ptr(), H.data_ptr(), _stream())
        return counts, H

    def penetrating_pairs(self, X, n: int):
        """Penetrating sphere-box pairs per particle (int32 [n])."""
        out = torch.empty(n, dtype=torch.int32, device=self.device)
        B.ct_penetrating_pairs(self.handle, X.data_ptr(), n, X.shape[1], out.data_ptr(), _stream())
        return out

    def step_mask(self, terms, n: int):
        """Eq. (3) per pick-place step ([K, ld] uint8) and the count of
        satisfied constraint terms per particle (int32 [n]), from ct_cost's
        terms (ct_step_mask)."""
        K = self.prob.skeleton.n_steps
        sm = torch.empty((K, terms.shape[1]), dtype=torch.uint8, device=self.device)
        cnt = torch.empty(n, dtype=torch.int32, device=self.device)
        B.ct_step_mask(self.handle, terms.data_ptr(), n, terms.shape[1], sm.data_ptr(), sm.shape[1], cnt.data_ptr(),
                       _stream())
        return sm, cnt

    def set_term_weights(self, W):
        """Per-particle term weights [n_terms][ld] (device, kept alive by the
        caller) for every later cost / gradient / step call, or None for the
        fixed lambda of Eq. (2)."""
        self._wts = W
        B.ct_set_term_weights(self.handle, None if W is None else W.data_ptr(), 0 if W is None else W.shape[1])

    def al_update(self, terms, n: int, rho: float, mu, W):
        """Method-of-multipliers step on the constraint weights (device)."""
        B.ct_al_update(self.handle, terms.data_ptr(), n, terms.shape[1], float(rho), mu.data_ptr(), W.data_ptr(),
                       _stream())

    def al_weights(self, terms, n: int, rho: float, mu, W):
        """PHR augmented-Lagrangian weights at the given terms (device)."""
        B.ct_al_weights(self.handle, terms.data_ptr(), n, terms.shape[1], float(rho), mu.data_ptr(), W.data_ptr(),
                        _stream())

    def cost_grad(self, X, n: int, weights=None):
        c = torch.empty(n, dtype=torch.float32, device=self.device)
        G = self.empty(n)
        B.ct_cost_grad(self.handle, X.data_ptr(), n, X.shape[1], c.data_ptr(), G.data_ptr(),
                       weights.data_ptr() if weights is not None else None, _stream())
        return c, G

    def adam_apply(self, X, M, V, G, n: int, t: int, adam: B.CtAdam, frozen=None):
        B.ct_adam_apply(self.handle, X.data_ptr(), M.data_ptr(), V.data_ptr(), G.data_ptr(), n, X.shape[1], t,
                        adam, frozen.data_ptr() if frozen is not None else None, _stream())

    def step(self, X, M, V, n: int, t: int, adam: B.CtAdam, frozen=None, cost=None, mask=None, first_sat=None):
        ptr = lambda a: a.data_ptr() if a is not None else None  # noqa: E731
        B.ct_step(self.handle, X.data_ptr(), M.data_ptr(), V.data_ptr(), n, X.shape[1], t, adam, ptr(frozen),
                  ptr(cost), ptr(mask), ptr(first_sat), _stream())

    def optimize(self, X, M, V, n: int, t0: int, iters: int, adam: B.CtAdam, frozen=None, cost=None, mask=None,
                 first_sat=None, stop_at_first: bool = False):
        ptr = lambda a: a.data_ptr() if a is not None else None  # noqa: E731
        B.ct_optimize(self.handle, X.data_ptr(), M.data_ptr(), V.data_ptr(), n, X.shape[1], t0, iters, adam,
                      ptr(frozen), ptr(cost), ptr(mask), ptr(first_sat), int(stop_at_first), _stream())

    def set_split(self, split: int):
        B.ct_set_split(self.handle, split)

    def get_split(self) -> int:
        return B.ct_get_split(self.handle)

    def autotune(self, X, n: int) -> int:
        return B.ct_autotune(self.handle, X.data_ptr(), n, X.shape[1], _stream())


class ParticleCost(torch.autograd.Function):
    """Per-particle cost J(x_i) of Eq. (2) as a differentiable torch op on a
    dimension-major particle buffer X [dim, ld].

    forward: ct_cost (nothing but X is saved);
    backward: ct_cost_grad with the incoming per-particle gradients as
    weights -- one kernel that recomputes forward kinematics of every
    configuration and motion waypoint and applies the hand-written adjoint.
    """

    @staticmethod
    def forward(ctx, X, gp: "GpuProblem", n: int):
        X = X.contiguous()
        c = torch.empty(n, dtype=torch.float32, device=X.device)
        B.ct_cost(gp.handle, X.data_ptr(), n, X.shape[1], c.data_ptr(), None, None, _stream())
        ctx.save_for_backward(X)
        ctx.gp, ctx.n = gp, n
        return c

    @staticmethod
    def backward(ctx, grad_c):
        (X,) = ctx.saved_tensors
        gp, n = ctx.gp, ctx.n
        w = grad_c.to(torch.float32).contiguous()
        G = torch.zeros_like(X)
        B.ct_cost_grad(gp.handle, X.data_ptr(), n, X.shape[1], None, G.data_ptr(), w.data_ptr(), _stream())
        return G, None, None


def particle_cost(gp: "GpuProblem", X: torch.Tensor, n: int) -> torch.Tensor:
    return ParticleCost.apply(X, gp, n)


def grasp_frozen(prob: I.Problem, device="cuda") -> torch.Tensor:
    """Frozen-dimension mask that fixes every step's grasp (gx, gy, gz, gyaw)
    after initialization: the paper samples grasps and keeps them fixed while
    placements and configurations are optimized (Sec. VII, Experimental
    Setup)."""
    f = torch.zeros(prob.dim, dtype=torch.uint8)
    for k in range(prob.skeleton.n_steps):
        f[I.STEP_DIM * k + 14:I.STEP_DIM * k + 18] = 1
    return f.to(device)


def sampler_frozen(prob: I.Problem, device="cuda") -> torch.Tensor:
    """Frozen-dimension mask of the conditional configuration sampler: every
    step's grasp and placement stay as the grasp and placement samplers drew
    them, only the configurations move."""
    f = grasp_frozen(prob, "cpu")
    for k in range(prob.skeleton.n_steps):
        f[I.STEP_DIM * k + 18:I.STEP_DIM * k + 21] = 1
    return f.to(device)


def default_adam(n: int, lr: float = 1e-2) -> B.CtAdam:
    """lr 1e-2, betas (0.9, 0.999), eps 1e-8, gradient scaled by 1/N_b (Eq. 4)."""
    return B.CtAdam(lr, 0.9, 0.999, 1e-8, 1.0 / n)


class GpuBatch:
    """Many skeletons bound to their own particle buffers, stepped together by
    one persistent launch per iteration (or, for comparison, one launch per
    skeleton)."""

    def __init__(self, problems: list, sizes: list[int], device="cuda", fixed_grasps: bool = True,
                 fixed_placements: bool = False):
        self.gps = [GpuProblem(p, device) for p in problems]
        self.sizes = list(sizes)
        self.device = torch.device(device)
        self.X = [g.empty(n) for g, n in zip(self.gps, sizes)]
        self.M = [g.empty(n) for g, n in zip(self.gps, sizes)]
        self.V = [g.empty(n) for g, n in zip(self.gps, sizes)]
        self.cost = [torch.empty(n, dtype=torch.float32, device=self.device) for n in sizes]
        self.mask = [torch.empty(n, dtype=torch.uint8, device=self.device) for n in sizes]
        self.first_sat = torch.full((len(sizes),), INT32_MAX, dtype=torch.int32, device=self.device)
        self.frozen = [sampler_frozen(p, self.device) if fixed_placements else
                       grasp_frozen(p, self.device) if fixed_grasps else None for p in problems]
        ptr = lambda a: a.data_ptr() if a is not None else None  # noqa: E731
        self.handle = B.ct_batch_create(
            [g.handle for g in self.gps], [x.data_ptr() for x in self.X], [m.data_ptr() for m in self.M],
            [v.data_ptr() for v in self.V], self.sizes, [x.shape[1] for x in self.X],
            [c.data_ptr() for c in self.cost], [m.data_ptr() for m in self.mask],
            [self.first_sat.data_ptr() + 4 * s for s in range(len(sizes))], [ptr(f) for f in self.frozen])

    def close(self):
        if getattr(self, "handle", None):
            B.ct_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def seed(self, seed: int, sampled: bool = False):
        """Uniform draws, or (sampled) the grasp and placement samplers'."""
        for s, (g, n) in enumerate(zip(self.gps, self.sizes)):
            draw = g.seed_sampled if sampled else g.seed_uniform
            draw(seed * 1000 + s, self.X[s], self.M[s], self.V[s], n)
        self.first_sat.fill_(INT32_MAX)

    def set_tuning(self, split=0, workgroups=0, persistent=True):
        B.ct_batch_set_tuning(self.handle, split, workgroups, int(persistent))

    def autotune(self):
        return B.ct_batch_autotune(self.handle, _stream())

    def step(self, t: int, adam: B.CtAdam):
        B.ct_batch_step(self.handle, t, adam, _stream())

    def optimize(self, t0: int, iters: int, adam: B.CtAdam):
        B.ct_batch_optimize(self.handle, t0, iters, adam, _stream())

    @property
    def particles(self) -> int:
        return sum(self.sizes)


@dataclass
class SolveResult:
    iters_budget: int
    first_sat_iter: int | None      # optimizer iterations before the first satisfying particle
    time_to_first_s: float | None   # GPU time from the start of initialization to the end of the
                                    # chunk of iterations that produced the first satisfying particle
    wall_s: float                   # host wall clock of the whole call
    n_satisfied: int                # satisfying particles at the last executed iterate
    solution: np.ndarray | None = None   # [n_satisfied, D] the satisfying particles (rows of X whose
                                         # mask is 1 after a stop at the first satisfying iterate)


INT32_MAX = 2 ** 31 - 1


def plain_solve(gp: GpuProblem, n: int, iters: int, seed: int, chunk: int = 10, stop_at_first: bool = True,
                adam: B.CtAdam | None = None, X=None, fixed_grasps: bool = True, init=None) -> SolveResult:
    """The plain method: uniform seeds (or `init(X, M, V)`, which enqueues
    another initializer and is timed with the solve), then Adam until the
    first satisfying particle or the iteration budget.  The whole budget is enqueued at once as
    replays of one captured `chunk`-step graph with a GPU event after each;
    with stop_at_first the device skips every step after the first satisfying
    iteration, so no host polling is needed.  Time to first = GPU time to the
    end of the chunk holding that iteration."""
    adam = adam or default_adam(n)
    frozen = grasp_frozen(gp.prob, gp.device) if fixed_grasps else None
    X = gp.empty(n) if X is None else X
    M, V = gp.empty(n), gp.empty(n)
    cost = torch.empty(n, dtype=torch.float32, device=gp.device)
    mask = torch.empty(n, dtype=torch.uint8, device=gp.device)
    flag = torch.full((1,), INT32_MAX, dtype=torch.int32, device=gp.device)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    if init is None:
        gp.seed_uniform(seed, X, M, V, n)
    else:
        init(X, M, V)
    events = []
    done = 0
    while done < iters:
        c = min(chunk, iters - done)
        gp.optimize(X, M, V, n, done, c, adam, frozen=frozen, cost=cost, mask=mask, first_sat=flag,
                    stop_at_first=stop_at_first)
        done += c
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        events.append(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    return _result(gp, X, mask, n, flag, iters, wall, start, events, chunk, stop_at_first)


def _result(gp, X, mask, n, flag, iters, wall, start, events, chunk, stopped) -> SolveResult:
    f = int(flag.item())
    if f == INT32_MAX:
        return SolveResult(iters, None, None, wall, int(mask.sum().item()))
    ttf = start.elapsed_time(events[min(f // chunk, len(events) - 1)]) / 1e3
    sol = gp.to_rows(X, n)[mask[:n].bool()].cpu().numpy() if stopped else None
    return SolveResult(iters, f, ttf, wall, int(mask.sum().item()), sol)


def al_solve(gp: GpuProblem, n: int, iters: int, seed: int, rho: float = 10.0, outer: int = 50, chunk: int = 10,
             adam: B.CtAdam | None = None, fixed_grasps: bool = True, init=None, mode: str = "phr") -> SolveResult:
    """The plain method with Lagrangian constraint weights: Adam on
    sum_c W_c J_c per particle.  Every `outer` iterations the multipliers
    take one method-of-multipliers step from the particles' current terms,
    mu <- max(0, mu + rho (J - eps)).
      mode "phr"  the PHR augmented Lagrangian: after every chunk the weights
                  are re-formed at the current terms,
                  W = lambda + max(0, mu + rho (J - eps)) (ct_al_weights),
                  the gradient weights of L = sum lambda J
                  + (1/2rho) sum (max(0, mu + rho g)^2 - mu^2);
      mode "dual" W = lambda + mu, fixed between multiplier steps (dual
                  ascent on the weights).
    Stops at the first satisfying particle (unweighted Eq. (3)) like
    plain_solve.  Uniform seeds, or `init(X, M, V)` (timed with the solve).
    `outer` must be a multiple of `chunk` (weights move between captured
    chunks)."""
    if mode not in ("phr", "dual"):
        raise ValueError(f"mode must be 'phr' or 'dual', not {mode!r}")
    if outer <= 0 or chunk <= 0 or outer % chunk:
        raise ValueError(f"outer ({outer}) must be a positive multiple of chunk ({chunk})")
    adam = adam or default_adam(n)
    frozen = grasp_frozen(gp.prob, gp.device) if fixed_grasps else None
    X, M, V = gp.empty(n), gp.empty(n), gp.empty(n)
    terms = gp.empty(n, rows=gp.n_terms)
    mu = torch.zeros_like(terms)
    W = torch.empty_like(terms)
    cost = torch.empty(n, dtype=torch.float32, device=gp.device)
    mask = torch.empty(n, dtype=torch.uint8, device=gp.device)
    flag = torch.full((1,), INT32_MAX, dtype=torch.int32, device=gp.device)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    if init is None:
        gp.seed_uniform(seed, X, M, V, n)
    else:
        init(X, M, V)
    gp.set_term_weights(None)
    B.ct_cost(gp.handle, X.data_ptr(), n, X.shape[1], cost.data_ptr(), terms.data_ptr(), None, _stream())
    gp.al_update(terms, n, 0.0, mu, W)            # W = lambda
    if mode == "phr":
        gp.al_weights(terms, n, rho, mu, W)       # W = lambda + max(0, rho (J - eps))
    gp.set_term_weights(W)
    events = []
    done = 0
    try:
        while done < iters:
            c = min(chunk, iters - done)
            gp.optimize(X, M, V, n, done, c, adam, frozen=frozen, cost=cost, mask=mask, first_sat=flag,
                        stop_at_first=True)
            done += c
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            events.append(e)
            update = done % outer == 0
            if done < iters and (update or mode == "phr"):
                B.ct_cost(gp.handle, X.data_ptr(), n, X.shape[1], cost.data_ptr(), terms.data_ptr(), None,
                          _stream())
                if update:
                    gp.al_update(terms, n, rho, mu, W)
                if mode == "phr":
                    gp.al_weights(terms, n, rho, mu, W)
        torch.cuda.synchronize()
    finally:
        gp.set_term_weights(None)
    wall = time.perf_counter() - t_wall
    return _result(gp, X, mask, n, flag, iters, wall, start, events, chunk, True)
