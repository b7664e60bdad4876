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

    def forward(self, feats, rows: int, seed: int, feat_of_row=None, draw=None) -> torch.Tensor:
        Y = torch.empty(rows, self.d_out, dtype=torch.float32, device=self.device)
        B.ct_mlp_forward(self.h, feats.data_ptr(), feats.shape[0], _ptr(feat_of_row), _ptr(draw), rows, seed,
                         Y.data_ptr(), _stream())
        return Y

    def backward(self, dY, rows: int):
        B.ct_mlp_backward(self.h, dY.data_ptr(), rows, _stream())

    def adam(self, lr: float = 1e-3, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        self.t += 1
        B.ct_mlp_adam(self.h, self.t, B.CtAdam(lr, beta1, beta2, eps, grad_scale), _stream())

    def imle_step(self, feats, feat_of_row, targets, n_draws: int, seed: int, lr: float = 1e-3, chosen=None,
                  loss=None):
        """One training step; returns the (device) loss tensor."""
        self.t += 1
        loss = self._loss if loss is None else loss
        B.ct_mlp_imle_step(self.h, feats.data_ptr(), feats.shape[0], feat_of_row.data_ptr(), targets.data_ptr(),
                           targets.shape[0], n_draws, seed, self.t, B.CtAdam(lr, 0.9, 0.999, 1e-8, 1.0),
                           loss.data_ptr(), _ptr(chosen), _stream())
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
    scene_of_row: np.ndarray   # [rows] int32
    n_sat: np.ndarray          # [rows] satisfied constraint count of each kept particle
    fully_satisfying: int      # kept particles that satisfy every constraint
    gpu_seconds: float


def collect(scene_seeds, robot_seed: int = 0, n: int = 8192, iters: int = 500, keep: int = 200,
            init_seed: int = 1000, log=None) -> Dataset:
    """Run the plain method (uniform seeds, fixed grasps, `iters` Adam steps)
    on the 4-object packing scene of every seed and keep each scene's `keep`
    best final particles.

    Reading: the method's converged particles are its particles at the end of
    the run; they are ranked by the number of constraints they satisfy
    (Eq. 3, per constraint), then by cost (Eq. 2), so fully satisfying
    particles come first and the rest are the nearest misses."""
    feats, rows, sc, nsat = [], [], [], []
    full = 0
    t_gpu = 0.0
    for j, s in enumerate(scene_seeds):
        prob = I.packing(robot_seed, int(s))
        gp = GpuProblem(prob)
        X, M, V = gp.empty(n), gp.empty(n), gp.empty(n)
        fz = grasp_frozen(prob, gp.device)
        t0 = time.perf_counter()
        gp.seed_uniform(init_seed + int(s), X, M, V, n)
        adam = default_adam(n)
        for t in range(0, iters, 50):       # replays of one captured 50-step graph
            gp.optimize(X, M, V, n, t, min(50, iters - t), adam, frozen=fz)
        cost, terms, _ = gp.cost(X, n, terms=True)
        torch.cuda.synchronize()
        t_gpu += time.perf_counter() - t0
        nc = prob.n_constraint_terms
        eps = torch.tensor(_tolerances(prob), dtype=torch.float32, device=gp.device)
        ok = (terms[:nc, :n] <= eps[:, None]).sum(0)
        c = torch.nan_to_num(cost[:n], nan=float("inf")).cpu().numpy()
        k = ok.cpu().numpy()
        order = np.lexsort((c, -k))[:keep]
        rows.append(gp.to_rows(X, n)[torch.from_numpy(order).to(gp.device)].cpu().numpy())
        nsat.append(k[order])
        full += int((k[order] == nc).sum())
        feats.append(I.scene_features(prob))
        sc.append(np.full(len(order), j, dtype=np.int32))
        gp.close()
        if log and (j + 1) % 50 == 0:
            log(f"collect: {j + 1}/{len(scene_seeds)} scenes, {full} fully satisfying kept")
    wrap = I.angle_dims(I.packing(robot_seed, int(scene_seeds[0])))
    return Dataset(np.stack(feats), wrap_angles(np.concatenate(rows), wrap), np.concatenate(sc),
                   np.concatenate(nsat), full, t_gpu)


def _tolerances(prob: I.Problem) -> list[float]:
    t = prob.tolerances
    per = [t.kin_pos, t.kin_rot, t.kin_pos, t.kin_rot, t.grasp, t.place, t.jlim, t.jlim, t.coll, t.coll, t.coll]
    return per * prob.skeleton.n_steps + [t.motion_coll] * prob.n_motion_terms


# --------------------------------------------------------------------------
# standardization (reading: per-dimension mean / standard deviation over the
# training set, angles wrapped first; features likewise; a floor keeps
# near-constant dimensions finite)


@dataclass
class Stats:
    feat_mean: np.ndarray
    feat_std: np.ndarray
    out_mean: np.ndarray
    out_std: np.ndarray

    @staticmethod
    def of(data: Dataset, floor: float = 1e-3) -> "Stats":
        return Stats(data.feats.mean(0), np.maximum(data.feats.std(0), floor), data.targets.mean(0),
                     np.maximum(data.targets.std(0), floor))

    def feats(self, f: np.ndarray) -> np.ndarray:
        return (f - self.feat_mean) / self.feat_std

    def targets(self, x: np.ndarray) -> np.ndarray:
        return (x - self.out_mean) / self.out_std


# --------------------------------------------------------------------------
# training


@dataclass
class TrainLog:
    losses: list = field(default_factory=list)   # mean loss per epoch
    steps: int = 0
    seconds: float = 0.0
    rows_per_s: float = 0.0
    flops: float = 0.0                            # matrix-core flops of all steps


def step_flops(dims, rows: int, n_draws: int) -> float:
    """Matrix-product flops of one IMLE step (2 per multiply-add): a forward
    over rows * n_draws draws, a forward over rows, and the two backward
    products (dW, dH) per layer; the first layer has no dH."""
    fwd = sum(2.0 * i * o for i, o in dims)
    bwd = sum(2.0 * i * o for i, o in dims) + sum(2.0 * i * o for i, o in dims[1:])
    return rows * (n_draws * fwd + fwd + bwd)


def train(mlp: GpuMlp, data: Dataset, stats: Stats, epochs: int = 20, batch: int = 4096, n_draws: int = 8,
          lr: float = 1e-3, seed: int = 0, log=None) -> TrainLog:
    """IMLE training (Li and Malik 2018) on standardized targets: each step
    draws n_draws noise vectors per target and fits the nearest output."""
    dev = mlp.device
    feats = torch.from_numpy(stats.feats(data.feats).astype(np.float32)).to(dev).contiguous()
    T = torch.from_numpy(stats.targets(data.targets).astype(np.float32)).to(dev).contiguous()
    S = torch.from_numpy(data.scene_of_row.astype(np.int32)).to(dev).contiguous()
    R = T.shape[0]
    steps_per_epoch = R // batch
    rng = np.random.default_rng(np.random.SeedSequence([0x7A1, seed]))
    out = TrainLog()
    losses = torch.zeros(epochs * steps_per_epoch, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(R)[:steps_per_epoch * batch].astype(np.int64)).to(dev)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            Tb = T.index_select(0, idx).contiguous()
            Sb = S.index_select(0, idx).contiguous()
            mlp.imle_step(feats, Sb, Tb, n_draws, seed * 1_000_003 + k, lr, loss=losses[k:k + 1])
            k += 1
        if log:
            torch.cuda.synchronize()
            log(f"epoch {ep + 1}/{epochs}: loss {losses[k - steps_per_epoch:k].mean().item():.4f}")
    torch.cuda.synchronize()
    out.seconds = time.perf_counter() - t0
    out.steps = k
    per = losses.view(epochs, steps_per_epoch).mean(1).cpu().numpy()
    out.losses = [float(v) for v in per]
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
    budget: int
    n: int


def compare(prop: Proposer, scene_seeds, n: int = 8192, budget: int = 500, robot_seed: int = 0,
            seed: int = 4242, log=None) -> Comparison:
    """Time to the first satisfying particle from uniform and from learned
    seeds on the same scenes, same budget, same optimizer; a learned run that
    finds nothing within the budget falls back to uniform seeds (its time is
    the failed learned run plus the uniform run)."""
    uni, lea, fb = [], [], []
    for s in scene_seeds:
        prob = I.packing(robot_seed, int(s))
        gp = GpuProblem(prob)
        pre = prop.prepare(prob)
        adam = default_adam(n)
        ru = plain_solve(gp, n, budget, seed=seed + int(s), adam=adam)
        rl = plain_solve(gp, n, budget, seed=seed + int(s), adam=adam,
                         init=lambda X, M, V: prop.seed(pre, seed + int(s), X, M, V, n))
        if rl.time_to_first_s is not None:
            f = rl.time_to_first_s
        elif ru.time_to_first_s is not None:
            f = rl.wall_s + ru.time_to_first_s
        else:
            f = None
        uni.append(ru)
        lea.append(rl)
        fb.append(f)
        gp.close()
        if log:
            log(f"scene {s}: uniform first {ru.first_sat_iter} ({ru.time_to_first_s}), "
                f"learned first {rl.first_sat_iter} ({rl.time_to_first_s}), sat at end {ru.satisfied}/{rl.satisfied}")
    return Comparison(list(scene_seeds), uni, lea, fb, budget, n)


def equal_rate_times(times_a, times_b):
    """Coverage of each method (fraction of scenes with a satisfying
    particle), the common rate r = min of the two, and the time at which each
    method has solved a fraction r of the scenes (None if r = 0)."""
    def cov(ts):
        return sum(t is not None for t in ts) / max(1, len(ts))

    ca, cb = cov(times_a), cov(times_b)
    r = min(ca, cb)
    if r == 0:
        return ca, cb, r, None, None

    def at(ts):
        k = max(1, math.ceil(r * len(ts)))
        return sorted(t for t in ts if t is not None)[k - 1]

    return ca, cb, r, at(times_a), at(times_b)
