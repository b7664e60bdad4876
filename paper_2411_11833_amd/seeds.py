"""Learned seed proposer: a BF16 multilayer perceptron, trained on the GPU by
implicit maximum likelihood on particles the plain method itself produced,
whose samples replace the uniform initializer; uniform seeding stays the
fallback (the paper initializes particles with samplers before optimizing
them, Sec. V "Particle Initialization").

Every step of training and sampling runs in the library's kernels
(``ct_mlp_*``: matrix-core products, GELU, noise, selection, Adam); this
module only prepares features and targets and drives the calls.  Readings
where the paper is silent (what the network sees, which particles count as
converged, standardization) are stated where they are used.
"""
from __future__ import annotations

import math
from fractions import Fraction
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from . import inputs as I
from .planner import GpuProblem, SolveResult, default_adam, grasp_frozen, plain_solve

D_FEAT = 120      # 12 objects x 10 features
D_NOISE = 32
HIDDEN = 512
DEPTH = 3


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


class GpuMlp:
    """Owns a ct_mlp handle.  Tensors passed in are CUDA tensors (float32 or
    int32, contiguous)."""

    def __init__(self, d_feat: int = D_FEAT, d_noise: int = D_NOISE, hidden: int = HIDDEN, depth: int = DEPTH,
                 d_out: int = 84, max_rows: int = 32768, device="cuda"):
        self.device = torch.device(device)
        self.d_feat, self.d_noise, self.hidden, self.depth, self.d_out = d_feat, d_noise, hidden, depth, d_out
        self.max_rows = max_rows
        self.h = B.ct_mlp_create(d_feat, d_noise, hidden, depth, d_out, max_rows)
        self.n_params = B.ct_mlp_info(self.h)
        self.t = 0
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            torch.cuda.synchronize()
            B.ct_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dims(self) -> list[tuple[int, int]]:
        d = [self.d_feat + self.d_noise] + [self.hidden] * self.depth + [self.d_out]
        return [(d[i], d[i + 1]) for i in range(self.depth + 1)]

    def set_params(self, p):
        p = torch.as_tensor(p, dtype=torch.float32).to(self.device).contiguous()
        assert p.numel() == self.n_params
        B.ct_mlp_set_params(self.h, p.data_ptr(), _stream())
        self.t = 0
        self._keep = p

    def params(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        B.ct_mlp_get_params(self.h, out.data_ptr(), _stream())
        return out

    def grads(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        B.ct_mlp_get_grads(self.h, out.data_ptr(), _stream())
        return out

    def noise(self, seed: int, rows: int, draw=None) -> torch.Tensor:
        out = torch.empty(rows, self.d_noise, dtype=torch.float32, device=self.device)
        B.ct_mlp_noise(self.h, seed, _ptr(draw), rows, out.data_ptr(), _stream())
        return out

    def forward(self, feats, rows: int, seed: int, feat_of_row=None, draw=None, keep: bool = True) -> torch.Tensor:
        """Y [rows, d_out]; keep=True keeps the activations for backward()."""
        Y = torch.empty(rows, self.d_out, dtype=torch.float32, device=self.device)
        fn = B.ct_mlp_forward if keep else B.ct_mlp_infer
        fn(self.h, feats.data_ptr(), feats.shape[0], _ptr(feat_of_row), _ptr(draw), rows, seed, Y.data_ptr(),
           _stream())
        return Y

    def backward(self, dY, rows: int):
        B.ct_mlp_backward(self.h, dY.data_ptr(), rows, _stream())

    def adam(self, lr: float = 1e-3, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        self.t += 1
        B.ct_mlp_adam(self.h, self.t, B.CtAdam(lr, beta1, beta2, eps, grad_scale), _stream())

    def imle_step(self, feats, feat_of_row, targets, n_draws: int, seed: int, lr: float = 1e-3, chosen=None,
                  loss=None, weights=None):
        """One training step; returns the (device) loss tensor."""
        self.t += 1
        loss = self._loss if loss is None else loss
        B.ct_mlp_imle_step(self.h, feats.data_ptr(), feats.shape[0], feat_of_row.data_ptr(), targets.data_ptr(),
                           _ptr(weights), targets.shape[0], n_draws, seed, self.t,
                           B.CtAdam(lr, 0.9, 0.999, 1e-8, 1.0), loss.data_ptr(), _ptr(chosen), _stream())
        return loss

    def sample(self, feats_row, seed: int, mean, std, lo, hi, wrap, X, M, V, n: int):
        B.ct_mlp_sample(self.h, feats_row.data_ptr(), seed, mean.data_ptr(), std.data_ptr(), lo.data_ptr(),
                        hi.data_ptr(), _ptr(wrap), X.data_ptr(), _ptr(M), _ptr(V), n, X.shape[1], _stream())


# --------------------------------------------------------------------------
# data: converged particles of the plain method


def wrap_angles(x: np.ndarray, wrap: np.ndarray) -> np.ndarray:
    """Angles (wrap = 1) into [-pi, pi)."""
    x = np.array(x, dtype=np.float64, copy=True)
    w = np.asarray(wrap, bool)
    x[..., w] = x[..., w] - 2 * math.pi * np.floor((x[..., w] + math.pi) / (2 * math.pi))
    return x


@dataclass
class Dataset:
    feats: np.ndarray          # [scenes, D_FEAT] raw scene features
    targets: np.ndarray        # [rows, dim] particles (angles wrapped)
    weights: np.ndarray        # [rows, dim] 1 where the entry's pick-place step satisfies all its constraints
    scene_of_row: np.ndarray   # [rows] int32
    n_sat: np.ndarray          # [rows] satisfied constraint count of each kept particle
    fully_satisfying: int      # kept particles that satisfy every constraint
    gpu_seconds: float


def packing_problem(seed: int, robot_seed: int = 0) -> I.Problem:
    return I.packing(robot_seed, seed)


def single_problem(seed: int, robot_seed: int = 0) -> I.Problem:
    return I.single_pick_place(robot_seed, seed)


def collect(scene_seeds, robot_seed: int = 0, n: int = 1024, iters: int = 1000, keep: int = 200,
            init_seed: int = 1000, log=None, proposer: "Proposer | None" = None, group: int = 64,
            make=packing_problem) -> Dataset:
    """Run the plain method (fixed grasps, `iters` Adam steps) on the problem
    `make(seed)` of every scene seed (default: 4-object packing), `group`
    scenes at a time in one persistent many-skeleton launch per iteration,
    and keep each scene's `keep` best final particles.

    Reading: the method's converged particles are its particles at the end of
    the run.  A pick-place step of a particle has converged when all of that
    step's constraints hold (Eq. 3); only converged steps are trusted as
    targets (weight 1 on their 21 entries, 0 elsewhere).  Particles are ranked
    by converged steps, then satisfied constraints, then cost (Eq. 2), and
    particles with no converged step are dropped.

    Runs start from uniform seeds, or with a proposer from its seeds (the
    next round of self-training: the method refines the proposer's seeds and
    its converged steps become new targets)."""
    from .planner import GpuBatch
    feats, rows, wts, sc, nsat = [], [], [], [], []
    full = 0
    t_gpu = 0.0
    seeds = [int(s) for s in scene_seeds]
    adam = default_adam(n)
    for g0 in range(0, len(seeds), group):
        chunk = seeds[g0:g0 + group]
        probs = [make(s, robot_seed) for s in chunk]
        gb = GpuBatch(probs, [n] * len(chunk))
        t0 = time.perf_counter()
        for j, (s, prob) in enumerate(zip(chunk, probs)):
            if proposer is None:
                gb.gps[j].seed_uniform(init_seed + s, gb.X[j], gb.M[j], gb.V[j], n)
            else:
                proposer.seed(proposer.prepare(prob), init_seed + s, gb.X[j], gb.M[j], gb.V[j], n)
        for t in range(0, iters, 50):       # replays of one captured 50-step graph
            gb.optimize(t, min(50, iters - t), adam)
        torch.cuda.synchronize()
        t_gpu += time.perf_counter() - t0
        for j, (s, prob) in enumerate(zip(chunk, probs)):
            gp = gb.gps[j]
            cost, terms, _ = gp.cost(gb.X[j], n, terms=True)
            nc = prob.n_constraint_terms
            steps, sat_count = gp.step_mask(terms, n)                                    # Eq. (3) per step
            c = torch.nan_to_num(cost[:n], nan=float("inf")).cpu().numpy()
            k = sat_count.cpu().numpy()
            st = steps[:, :n].cpu().numpy().astype(bool)
            ns = st.sum(0)
            order = np.lexsort((c, -k, -ns))[:keep]
            order = order[ns[order] > 0]
            rows.append(gp.to_rows(gb.X[j], n)[torch.from_numpy(order).to(gp.device)].cpu().numpy())
            wts.append(np.repeat(st[:, order].T.astype(np.float32), I.STEP_DIM, axis=1))
            nsat.append(k[order])
            full += int((k[order] == nc).sum())
            feats.append(I.scene_features(prob))
            sc.append(np.full(len(order), g0 + j, dtype=np.int32))
        gb.close()
        for g in gb.gps:
            g.close()
        if log:
            log(f"collect: {g0 + len(chunk)}/{len(seeds)} scenes, {sum(len(r) for r in rows)} particles kept, "
                f"{full} fully satisfying")
    wrap = I.angle_dims(make(seeds[0], robot_seed))
    return Dataset(np.stack(feats), wrap_angles(np.concatenate(rows), wrap), np.concatenate(wts),
                   np.concatenate(sc), np.concatenate(nsat), full, t_gpu)


def collect_steps(scene_seeds, robot_seed: int = 0, n: int = 1024, iters: int = 1000, keep: int = 64,
                  init_seed: int = 3000, log=None, group: int = 64) -> Dataset:
    """First-round targets from the method on each pick-place step alone:
    for every packing scene and every step k, the one-step skeleton that
    moves object k (the other objects stay where they are, as obstacles) is
    solved by the plain method (uniform seeds, fixed grasps), `group`
    skeletons per persistent launch.  Particles that satisfy every
    constraint of their one-step problem (Eq. 3) become targets for step k of
    the packing particle: their 21 entries go to step k's block with weight
    1, the other blocks have weight 0.  At most `keep` per step, lowest cost
    first.  (The paper's own initializer likewise composes per-action
    samplers, Sec. V.)"""
    from .planner import GpuBatch
    seeds = [int(s) for s in scene_seeds]
    subs = []   # (scene index, step, problem)
    packs = []
    for j, s in enumerate(seeds):
        pk = I.packing(robot_seed, s)
        packs.append(pk)
        for k in range(pk.skeleton.n_steps):
            sk = I.Skeleton(object_of_step=np.array([pk.skeleton.object_of_step[k]], dtype=np.int32))
            subs.append((j, k, I.Problem(pk.robot, pk.scene, sk)))
    D = packs[0].dim
    rows, wts, sc, nsat = [], [], [], []
    t_gpu = 0.0
    adam = default_adam(n)
    for g0 in range(0, len(subs), group):
        chunk = subs[g0:g0 + group]
        gb = GpuBatch([p for _, _, p in chunk], [n] * len(chunk))
        t0 = time.perf_counter()
        for i, (j, k, p) in enumerate(chunk):
            gb.gps[i].seed_uniform(init_seed + 8 * seeds[j] + k, gb.X[i], gb.M[i], gb.V[i], n)
        for t in range(0, iters, 50):
            gb.optimize(t, min(50, iters - t), adam)
        torch.cuda.synchronize()
        t_gpu += time.perf_counter() - t0
        for i, (j, k, p) in enumerate(chunk):
            gp = gb.gps[i]
            cost, _, m = gp.cost(gb.X[i], n, terms=False)
            ok = m[:n].bool().cpu().numpy()
            c = torch.nan_to_num(cost[:n], nan=float("inf")).cpu().numpy()
            idx = np.nonzero(ok)[0]
            idx = idx[np.argsort(c[idx], kind="stable")][:keep]
            if len(idx) == 0:
                continue
            blk = gp.to_rows(gb.X[i], n)[torch.from_numpy(idx).to(gp.device)].cpu().numpy()
            r = np.zeros((len(idx), D))
            w = np.zeros((len(idx), D), dtype=np.float32)
            r[:, I.STEP_DIM * k:I.STEP_DIM * (k + 1)] = blk
            w[:, I.STEP_DIM * k:I.STEP_DIM * (k + 1)] = 1.0
            rows.append(r)
            wts.append(w)
            sc.append(np.full(len(idx), j, dtype=np.int32))
            nsat.append(np.full(len(idx), I.TERMS_PER_STEP))
        gb.close()
        for g in gb.gps:
            g.close()
        if log:
            log(f"collect (one step at a time): {g0 + len(chunk)}/{len(subs)} skeletons, "
                f"{sum(len(r) for r in rows)} converged steps")
    wrap = I.angle_dims(packs[0])
    if not rows:
        raise RuntimeError("no one-step skeleton produced a satisfying particle")
    return Dataset(np.stack([I.scene_features(p) for p in packs]), wrap_angles(np.concatenate(rows), wrap),
                   np.concatenate(wts), np.concatenate(sc), np.concatenate(nsat), 0, t_gpu)


def merge(a: Dataset, b: Dataset) -> Dataset:
    """Two collections over the same scene list (b's scene indices follow
    a's feature rows)."""
    off = a.feats.shape[0]
    return Dataset(np.concatenate([a.feats, b.feats]), np.concatenate([a.targets, b.targets]),
                   np.concatenate([a.weights, b.weights]), np.concatenate([a.scene_of_row, b.scene_of_row + off]),
                   np.concatenate([a.n_sat, b.n_sat]), a.fully_satisfying + b.fully_satisfying,
                   a.gpu_seconds + b.gpu_seconds)


# --------------------------------------------------------------------------
# standardization (reading: per-dimension mean / standard deviation over the
# trusted entries of the training set, angles wrapped first; features
# likewise over the scenes; a floor keeps near-constant dimensions finite)


@dataclass
class Stats:
    feat_mean: np.ndarray
    feat_std: np.ndarray
    out_mean: np.ndarray
    out_std: np.ndarray

    @staticmethod
    def of(data: Dataset, floor: float = 1e-3) -> "Stats":
        w = data.weights.astype(np.float64)
        cnt = np.maximum(w.sum(0), 1.0)
        mean = (w * data.targets).sum(0) / cnt
        std = np.sqrt((w * (data.targets - mean) ** 2).sum(0) / cnt)
        return Stats(data.feats.mean(0), np.maximum(data.feats.std(0), floor), mean, np.maximum(std, floor))

    def feats(self, f: np.ndarray) -> np.ndarray:
        return (f - self.feat_mean) / self.feat_std

    def targets(self, x: np.ndarray) -> np.ndarray:
        return (x - self.out_mean) / self.out_std


# --------------------------------------------------------------------------
# training


@dataclass
class TrainLog:
    losses: list = field(default_factory=list)   # mean loss per tenth of the run
    steps: int = 0
    seconds: float = 0.0
    rows_per_s: float = 0.0
    flops: float = 0.0                            # matrix-core flops of all steps


def step_flops(dims, rows: int, n_draws: int) -> float:
    """Matrix-product flops of one IMLE step (2 per multiply-add): a forward
    over rows * n_draws draws, the hidden layers again over the rows kept
    (their outputs come from the first forward), and the two backward
    products (dW, dH) per layer; the first layer has no dH."""
    fwd = sum(2.0 * i * o for i, o in dims)
    hid = sum(2.0 * i * o for i, o in dims[:-1])
    bwd = sum(2.0 * i * o for i, o in dims) + sum(2.0 * i * o for i, o in dims[1:])
    return rows * (n_draws * fwd + hid + bwd)


def train(mlp: GpuMlp, data: Dataset, stats: Stats, steps: int = 2000, batch: int = 4096, n_draws: int = 8,
          lr: float = 1e-3, seed: int = 0, log=None) -> TrainLog:
    """IMLE training (Li and Malik 2018) on standardized targets: each step
    draws n_draws noise vectors per target and fits the nearest output, on
    the trusted entries only."""
    dev = mlp.device
    feats = torch.from_numpy(stats.feats(data.feats).astype(np.float32)).to(dev).contiguous()
    T = torch.from_numpy(stats.targets(data.targets).astype(np.float32)).to(dev).contiguous()
    W = torch.from_numpy(data.weights.astype(np.float32)).to(dev).contiguous()
    S = torch.from_numpy(data.scene_of_row.astype(np.int32)).to(dev).contiguous()
    R = T.shape[0]
    rng = np.random.default_rng(np.random.SeedSequence([0x7A1, seed]))
    out = TrainLog()
    losses = torch.zeros(steps, dtype=torch.float32, device=dev)
    # batches drawn as consecutive slices of a fresh permutation per pass
    order = np.concatenate([rng.permutation(R) for _ in range((steps * batch) // R + 1)])[:steps * batch]
    order = torch.from_numpy(order.astype(np.int64)).to(dev)
    # the batches of CHUNK steps are gathered at once (one copy per chunk,
    # not three per step); a step's batch is then a contiguous slice
    CHUNK = 64
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        if k % CHUNK == 0:
            idx = order[k * batch:min(k + CHUNK, steps) * batch]
            Tc, Wc, Sc = T.index_select(0, idx), W.index_select(0, idx), S.index_select(0, idx)
        r0 = (k % CHUNK) * batch
        Tb, Wb, Sb = Tc[r0:r0 + batch], Wc[r0:r0 + batch], Sc[r0:r0 + batch]
        mlp.imle_step(feats, Sb, Tb, n_draws, seed * 1_000_003 + k, lr, loss=losses[k:k + 1], weights=Wb)
        if log and (k + 1) % max(1, steps // 10) == 0:
            log(f"step {k + 1}/{steps}: loss {losses[max(0, k - 49):k + 1].mean().item():.4f}")
    torch.cuda.synchronize()
    out.seconds = time.perf_counter() - t0
    out.steps = steps
    per = losses.view(10, -1).mean(1).cpu().numpy() if steps % 10 == 0 else losses.cpu().numpy()
    out.losses = [float(v) for v in per]   # mean loss per tenth of the run
    out.rows_per_s = k * batch / out.seconds
    out.flops = k * step_flops(mlp.dims, batch, n_draws)
    return out


# --------------------------------------------------------------------------
# seeding and the learned-vs-uniform comparison


class Proposer:
    """A trained network plus its standardization, ready to seed problems."""

    def __init__(self, mlp: GpuMlp, stats: Stats):
        self.mlp, self.stats = mlp, stats
        dev = mlp.device
        self._mean = torch.from_numpy(stats.out_mean.astype(np.float32)).to(dev)
        self._std = torch.from_numpy(stats.out_std.astype(np.float32)).to(dev)

    def prepare(self, prob: I.Problem):
        """Device copies of one problem's features and bounds (scene
        description, uploaded before any timing)."""
        dev = self.mlp.device
        f = torch.from_numpy(self.stats.feats(I.scene_features(prob)).astype(np.float32)).to(dev)
        lo, hi = prob.bounds()
        return (f, torch.from_numpy(lo.astype(np.float32)).to(dev), torch.from_numpy(hi.astype(np.float32)).to(dev),
                torch.from_numpy(I.angle_dims(prob)).to(dev))

    def seed(self, prepared, seed: int, X, M, V, n: int):
        f, lo, hi, wrap = prepared
        self.mlp.sample(f, seed, self._mean, self._std, lo, hi, wrap, X, M, V, n)


@dataclass
class Comparison:
    scenes: list
    uniform: list            # SolveResult per scene
    learned: list            # SolveResult per scene (learned seeds only)
    learned_fallback: list   # time to first with the uniform fallback after an unsolved learned run (s or None)
    uniform_steps: list      # per scene: fraction of (particle, step) pairs whose step holds at the end
    learned_steps: list
    uniform_best: list       # per scene: most converged steps in one particle at the end
    learned_best: list
    budget: int
    n: int


def step_convergence(gp: GpuProblem, X, n: int) -> tuple[float, int]:
    """Fraction of (particle, pick-place step) pairs whose step satisfies all
    its constraints (Eq. 3 restricted to the step), and the largest number of
    such steps in one particle."""
    _, terms, _ = gp.cost(X, n, terms=True)
    steps, _ = gp.step_mask(terms, n)
    per = steps[:, :n].sum(0, dtype=torch.int32)
    return float(steps[:, :n].float().mean().item()), int(per.max().item())


def compare(prop: Proposer, scene_seeds, n: int = 8192, budget: int = 500, robot_seed: int = 0,
            seed: int = 4242, log=None, make=packing_problem) -> Comparison:
    """Time to the first satisfying particle from uniform and from learned
    seeds on the same scenes, same budget, same optimizer; a learned run that
    finds nothing within the budget falls back to uniform seeds (its time is
    the failed learned run plus the uniform run).  Also the per-step
    convergence at the end of each run."""
    out = Comparison(list(scene_seeds), [], [], [], [], [], [], [], budget, n)
    for s in scene_seeds:
        prob = make(int(s), robot_seed)
        gp = GpuProblem(prob)
        pre = prop.prepare(prob)
        adam = default_adam(n)
        X = gp.empty(n)
        ru = plain_solve(gp, n, budget, seed=seed + int(s), adam=adam, X=X)
        su = step_convergence(gp, X, n)
        rl = plain_solve(gp, n, budget, seed=seed + int(s), adam=adam, X=X,
                         init=lambda X_, M_, V_: prop.seed(pre, seed + int(s), X_, M_, V_, n))
        sl = step_convergence(gp, X, n)
        if rl.time_to_first_s is not None:
            f = rl.time_to_first_s
        elif ru.time_to_first_s is not None:
            f = rl.wall_s + ru.time_to_first_s
        else:
            f = None
        out.uniform.append(ru)
        out.learned.append(rl)
        out.learned_fallback.append(f)
        out.uniform_steps.append(su[0])
        out.learned_steps.append(sl[0])
        out.uniform_best.append(su[1])
        out.learned_best.append(sl[1])
        gp.close()
        if log:
            log(f"scene {s}: first satisfying iteration uniform {ru.first_sat_iter} / learned {rl.first_sat_iter}; "
                f"converged steps uniform {su[0]:.4f} (best {su[1]}) / learned {sl[0]:.4f} (best {sl[1]})")
    return out


def equal_rate_times(times_a, times_b):
    """Coverage of each method (fraction of scenes with a satisfying
    particle), the common rate r = min of the two, and the time at which each
    method has solved a fraction r of the scenes (None if r = 0)."""
    # The rate is kept as an exact fraction: in floating point, r * len(ts)
    # can round above the number of solved scenes (7/25 * 25 > 7) and index
    # past the sorted times.
    def cov(ts):
        return Fraction(sum(t is not None for t in ts), max(1, len(ts)))

    fa, fb = cov(times_a), cov(times_b)
    r = min(fa, fb)
    if r == 0:
        return float(fa), float(fb), 0.0, None, None

    def at(ts):
        k = max(1, math.ceil(r * len(ts)))
        return sorted(t for t in ts if t is not None)[k - 1]

    return float(fa), float(fb), float(r), at(times_a), at(times_b)
