"""FP64 CPU oracle of the particle cost / gradient / Adam step.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.  It shares no code with the HIP path.

Every quantity is written as its plain definition with batched PyTorch CPU
float64 ops (4x4 homogeneous transforms, explicit per-box loops); the
gradient is ``torch.autograd`` of that definition, i.e. the exact derivative of
the oracle's own cost.  References are to the paper (Shen et al.,
"Differentiable GPU-Parallelized Task and Motion Planning"):

* particle, constraint cost J_c, tolerance eps_c ............ Sec. IV-A
* weighted relaxation  J(x) = sum lambda_c J_c + soft costs ... Eq. (2)
* satisfaction test  AND_c J_c <= eps_c ...................... Eq. (3)
* batch objective (mean over the N_b particles) ............. Eq. (4)
* plan-skeleton feasibility heuristic H ...................... Eq. (5)
* Adam on that objective ..................................... Sec. IV-B
* per-particle (augmented-Lagrangian) term weights and the
  method-of-multipliers update ............................... Sec. IV-B (optimizers the method
                                                                admits), Sec. "Limitations"
* Kin(q,o,g,p): FK(q) = p * g, pose error .................... Sec. III, App. listing of example cost functions
* distance from bounds, pairwise object distance ............. App. listing of example cost functions
* weights (1, kin-rot 5, stable place 2), tolerances ........ App. "Cost Weights", "Constraint Tolerances"
* spheres vs oriented boxes .................................. App. "Collision Representation"
* robot self-collision (spheres of non-adjacent links) ....... Sec. IV-B "Parallelizing on GPUs",
                                                                App. "Constraint Tolerances"

Readings where the paper is silent are listed in the design notes (robot
DH form, pose-error form, grasp box, containment, collision hinge, box sets).

Parity pins live in ``tests/test_oracle_pins.py``.  One function is parity
unpinned against the paper itself: the paper prints no worked numeric
example, so only closed forms, brute force, finite differences and library
routines pin the oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from paper_2411_11833_amd.inputs import Problem, STEP_DIM, TERMS_PER_STEP

DT = torch.float64

__all__ = [
    "rz", "rx", "trans", "fk_frames", "box_sdf", "sphere_box_penalty", "pose_error",
    "dist_from_bounds", "pairwise_dist_sum", "grasp_tf", "place_tf", "evaluate",
    "Evaluation", "terms", "cost", "mask", "cost_and_grad", "adam_step", "margins",
    "weights_vector", "tolerance_vector", "place_z", "feasibility", "self_pairs", "self_collision",
    "weighted_cost_and_grad", "al_update", "phr_weights", "phr_lagrangian", "penetrating_pairs",
]


# ----------------------------------------------------------------------------
# homogeneous transforms (batched over the leading dims of the argument)


def _t(x):
    return torch.as_tensor(x, dtype=DT)


def rz(t: torch.Tensor) -> torch.Tensor:
    """Rotation about z by angle t, as a 4x4 transform."""
    t = _t(t)
    c, s, z, o = torch.cos(t), torch.sin(t), torch.zeros_like(t), torch.ones_like(t)
    return torch.stack([c, -s, z, z, s, c, z, z, z, z, o, z, z, z, z, o], -1).reshape(*t.shape, 4, 4)


def rx(t: torch.Tensor) -> torch.Tensor:
    """Rotation about x by angle t, as a 4x4 transform."""
    t = _t(t)
    c, s, z, o = torch.cos(t), torch.sin(t), torch.zeros_like(t), torch.ones_like(t)
    return torch.stack([o, z, z, z, z, c, -s, z, z, s, c, z, z, z, z, o], -1).reshape(*t.shape, 4, 4)


def trans(x, y, z) -> torch.Tensor:
    """Pure translation by (x, y, z), as a 4x4 transform."""
    x, y, z = torch.broadcast_tensors(_t(x), _t(y), _t(z))
    o, n = torch.ones_like(x), torch.zeros_like(x)
    return torch.stack([o, n, n, x, n, o, n, y, n, n, o, z, n, n, n, o], -1).reshape(*x.shape, 4, 4)


def fk_frames(robot, q: torch.Tensor) -> list[torch.Tensor]:
    """Forward kinematics FK(q) of a standard-DH serial arm.

    Frame i = frame (i-1) * Rz(q_i + theta0_i) * Tz(d_i) * Tx(a_i) * Rx(alpha_i),
    frame 0 is the world (base at the origin), and the tool frame is
    frame 7 * Tz(tool_d).  Returns [F_0, F_1, ..., F_7, F_ee], each [B, 4, 4].
    """
    B = q.shape[0]
    F = torch.eye(4, dtype=DT).expand(B, 4, 4)
    frames = [F]
    for i in range(robot.dh.shape[0]):
        a, al, d, th0 = (float(v) for v in robot.dh[i])
        zero = torch.zeros(B, dtype=DT)
        A = rz(q[:, i] + th0) @ trans(zero, zero, zero + d) @ trans(zero + a, zero, zero) @ rx(zero + al)
        F = F @ A
        frames.append(F)
    zero = torch.zeros(B, dtype=DT)
    frames.append(F @ trans(zero, zero, zero + robot.tool_d))
    return frames


def apply(T: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """World coordinates of points p [..., S, 3] given in the frame T [..., 4, 4]."""
    return (T[..., None, :3, :3] @ p[..., None]).squeeze(-1) + T[..., None, :3, 3]


def grasp_tf(g: torch.Tensor) -> torch.Tensor:
    """Top-down grasp G = Trans(gx, gy, gz) Rz(gyaw) Rx(pi): the tool pose in
    the object frame, tool z-axis pointing down."""
    return trans(g[:, 0], g[:, 1], g[:, 2]) @ rz(g[:, 3]) @ rx(torch.full_like(g[:, 3], math.pi))


def place_z(prob: Problem, obj: int) -> float:
    """Height of a stably placed object's centre: table top plus half height."""
    tb = prob.scene.table
    return float(tb[2] + tb[6] + prob.scene.objects[obj, 6])


def place_tf(rho: torch.Tensor, z: float) -> torch.Tensor:
    """4-DOF placement P = Trans(px, py, z) Rz(pyaw) on the table top."""
    return trans(rho[:, 0], rho[:, 1], torch.full_like(rho[:, 0], z)) @ rz(rho[:, 2])


def box_tf(b: np.ndarray) -> torch.Tensor:
    """Pose of a yaw-only box given as (cx, cy, cz, yaw, hx, hy, hz)."""
    return trans(float(b[0]), float(b[1]), float(b[2])) @ rz(torch.tensor(float(b[3]), dtype=DT))


# ----------------------------------------------------------------------------
# primitive distances


def box_sdf(c: torch.Tensor, T_box: torch.Tensor, half: torch.Tensor) -> torch.Tensor:
    """Signed distance from points c [B, S, 3] to an oriented box with pose
    T_box [B or 1, 4, 4] and half extents half [3]: with p the point in the box
    frame and u = |p| - half, sdf = ||max(u, 0)|| + min(max_i u_i, 0)."""
    R = T_box[..., :3, :3]
    t = T_box[..., :3, 3]
    p = ((c - t[..., None, :])[..., None, :] @ R[..., None, :, :]).squeeze(-2)   # R^T (c - t)
    u = p.abs() - half
    outside = torch.linalg.vector_norm(torch.clamp(u, min=0.0), dim=-1)
    inside = torch.clamp(u.max(dim=-1).values, max=0.0)
    return outside + inside


def sphere_box_penalty(c: torch.Tensor, r: torch.Tensor, T_box: torch.Tensor, half) -> torch.Tensor:
    """Per-sphere penetration max(0, r - sdf) [B, S] of spheres vs one box."""
    return torch.clamp(r - box_sdf(c, T_box, _t(half)), min=0.0)


def pose_error(Ta: torch.Tensor, Tb: torch.Tensor):
    """(position error, rotation error) between two poses: the Euclidean
    distance of the origins and the geodesic angle of R_a^T R_b,
    theta = atan2(||vee(R - R^T)|| / 2, (trace R - 1) / 2) in [0, pi]."""
    pos = torch.linalg.vector_norm(Ta[..., :3, 3] - Tb[..., :3, 3], dim=-1)
    R = Ta[..., :3, :3].transpose(-1, -2) @ Tb[..., :3, :3]
    w = torch.stack([R[..., 2, 1] - R[..., 1, 2], R[..., 0, 2] - R[..., 2, 0],
                     R[..., 1, 0] - R[..., 0, 1]], -1) / 2
    cos_t = (R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2] - 1) / 2
    rot = torch.atan2(torch.linalg.vector_norm(w, dim=-1), cos_t)
    return pos, rot


def dist_from_bounds(v: torch.Tensor, lo, hi) -> torch.Tensor:
    """Euclidean distance of v [..., d] from the box [lo, hi]; zero inside."""
    lo, hi = _t(lo), _t(hi)
    below = torch.clamp(lo - v, min=0.0)
    above = torch.clamp(v - hi, min=0.0)
    return torch.linalg.vector_norm(below + above, dim=-1)


def pairwise_dist_sum(p: torch.Tensor) -> torch.Tensor:
    """Sum over unordered pairs i < j of ||p_i - p_j|| for p [B, n, 3]."""
    n = p.shape[1]
    total = torch.zeros(p.shape[0], dtype=DT)
    for i in range(n):
        for j in range(i + 1, n):
            total = total + torch.linalg.vector_norm(p[:, i] - p[:, j], dim=-1)
    return total


# ----------------------------------------------------------------------------
# the CSP of one pick-place skeleton


@dataclass
class Evaluation:
    terms: torch.Tensor      # [B, n_terms] unweighted J_c / soft costs
    cost: torch.Tensor       # [B] weighted sum, Eq. (2)
    kinks: list              # tensors [B] of distances to nonsmooth points (if requested)
    flip_lo: list            # per constraint term: [B] distance inside an eps = 0 bound
    pair_args: list = None   # hinge arguments r - sdf [B, S] of every sphere-box pair set (if requested)


def weights_vector(prob: Problem) -> np.ndarray:
    w, K = prob.weights, prob.skeleton.n_steps
    per = [w.kin_pos, w.kin_rot, w.kin_pos, w.kin_rot, w.grasp, w.place, w.jlim, w.jlim,
           w.coll, w.coll, w.coll]
    out = per * K + [w.motion_coll] * prob.n_motion_terms + [w.self_coll] * prob.n_self_terms
    if prob.skeleton.goal_cost:
        out.append(w.goal)
    if prob.skeleton.waypoints > 0:
        out.append(w.traj_len)
    return np.array(out, dtype=np.float64)


def tolerance_vector(prob: Problem) -> np.ndarray:
    """Tolerances of the constraint terms (soft costs have none)."""
    e, K = prob.tolerances, prob.skeleton.n_steps
    per = [e.kin_pos, e.kin_rot, e.kin_pos, e.kin_rot, e.grasp, e.place, e.jlim, e.jlim,
           e.coll, e.coll, e.coll]
    return np.array(per * K + [e.motion_coll] * prob.n_motion_terms + [e.self_coll] * prob.n_self_terms,
                    dtype=np.float64)


def _robot_spheres(prob: Problem, frames):
    """World centres [B, S, 3] and radii [S] of the robot spheres."""
    r = prob.robot
    cs = []
    for s in range(r.spheres.shape[0]):
        F = frames[int(r.sphere_link[s])]
        cs.append(apply(F, _t(r.spheres[s:s + 1, :3]).expand(F.shape[0], 1, 3)))
    return torch.cat(cs, 1), _t(r.spheres[:, 3])


def _collision(c, rad, boxes, kinks, want_kinks, pair_args=None):
    """Sum over spheres and boxes of max(0, r - sdf); records the kink
    distances of the hinge and of the interior max when asked, and the hinge
    arguments themselves into pair_args when given."""
    total = torch.zeros(c.shape[0], dtype=DT)
    for T, h in boxes:
        half = _t(h)
        sdf = box_sdf(c, T, half)
        arg = rad - sdf
        total = total + torch.clamp(arg, min=0.0).sum(-1)
        if pair_args is not None:
            pair_args.append(arg.detach())
        if want_kinks:
            with torch.no_grad():
                kinks.append(arg.abs().min(-1).values)
                R = T[..., :3, :3]
                t = T[..., :3, 3]
                p = ((c - t[..., None, :])[..., None, :] @ R[..., None, :, :]).squeeze(-2)
                u = p.abs() - half
                top2 = torch.topk(u, 2, dim=-1).values
                inside_active = (u.max(-1).values <= 0) & (arg > 0)
                gap = torch.where(inside_active, top2[..., 0] - top2[..., 1],
                                  torch.full_like(arg, math.inf))
                ax = u.argmax(-1, keepdim=True)
                pa = torch.where(inside_active, p.gather(-1, ax).squeeze(-1).abs(),
                                 torch.full_like(arg, math.inf))
                kinks.append(torch.minimum(gap, pa).min(-1).values)
    return total


def self_pairs(sphere_link) -> tuple[np.ndarray, np.ndarray]:
    """Index pairs (a, b), a < b, of robot spheres whose rigid segments are
    neither the same nor neighbours in the chain (|link_a - link_b| >= 2;
    segments 1..7 are the links, 8 the tool).  Neighbouring segments meet at
    a joint, where their spheres overlap by construction."""
    L = np.asarray(sphere_link, dtype=np.int64)
    a, b = np.triu_indices(L.size, k=1)
    keep = np.abs(L[a] - L[b]) >= 2
    return a[keep], b[keep]


def self_collision(c, rad, sphere_link, kinks=None, want_kinks=False):
    """Self-penetration of one configuration: sum over the pairs of
    ``self_pairs`` of max(0, r_a + r_b - |c_a - c_b|), for world centres c
    [B, S, 3] and radii rad [S].  Returns (penalty [B], the largest hinge
    argument [B]; minus it is how far the closest pair is from touching)."""
    ia, ib = self_pairs(sphere_link)
    ia, ib = torch.as_tensor(ia), torch.as_tensor(ib)
    d = torch.linalg.vector_norm(c[:, ia] - c[:, ib], dim=-1)
    arg = rad[ia] + rad[ib] - d
    if want_kinks:
        with torch.no_grad():
            kinks.append(arg.abs().min(-1).values)
            kinks.append(d.min(-1).values)
    return torch.clamp(arg, min=0.0).sum(-1), arg.detach().max(-1).values


def evaluate(prob: Problem, X: torch.Tensor, want_kinks: bool = False, want_pairs: bool = False) -> Evaluation:
    """All terms of Eq. (2) for particles X [B, dim] (float64).

    Term order per pick-place step k (object o = object_of_step[k]):
      0 Kin position error at the pick   |FK(q_g) - P0_o G(g)|           (lambda 1, eps 5 mm)
      1 Kin rotation error at the pick                                      (lambda 5, eps 0.05 rad)
      2 Kin position error at the place  |FK(q_p) - P(rho) G(g)|         (lambda 1, eps 5 mm)
      3 Kin rotation error at the place                                     (lambda 5, eps 0.05 rad)
      4 Grasp: distance of the grasp position from the valid grasp box     (lambda 1, eps 0)
      5 StablePlace: sum over footprint corners of the distance from the
        region                                                              (lambda 2, eps 1 mm)
      6/7 joint-limit distance of q_g / q_p                                 (lambda 1, eps 0)
      8 CFreeHold at q_g: robot + held-object spheres vs the step's boxes   (lambda 1, eps 1 mm)
      9 the same at q_p                                                     (lambda 1, eps 1 mm)
      10 CFreePlace: object spheres at P(rho) vs the step's boxes          (lambda 1, eps 1 mm)
    then, with motion, one collision term per transition, then, with
    self-collision, one self-penetration term per key configuration (q_g of
    step k at 2k, q_p at 2k + 1; lambda 1, eps 0), then the soft costs: the
    goal's pairwise placed-object distance and the trajectory length.

    The boxes of step k are the table, the obstacles, objects the skeleton
    never moves, and every other moved object: at its placement if placed
    by an earlier step, else at its initial pose.  The object of step k is
    held (or about to be) and is not an obstacle to the robot in its own step.
    """
    r, sc, sk = prob.robot, prob.scene, prob.skeleton
    K = sk.n_steps
    B = X.shape[0]
    kinks: list = []
    flip_lo: list = []
    moved = [int(o) for o in sk.object_of_step]
    P0 = [box_tf(sc.objects[o]) for o in moved]
    rho = [X[:, STEP_DIM * k + 18:STEP_DIM * k + 21] for k in range(K)]
    P = [place_tf(rho[k], place_z(prob, moved[k])) for k in range(K)]

    static = [(box_tf(sc.table)[None], sc.table[4:7])]
    static += [(box_tf(b)[None], b[4:7]) for b in sc.obstacles]
    static += [(box_tf(sc.objects[o])[None], sc.objects[o, 4:7])
               for o in range(sc.objects.shape[0]) if o not in moved]

    def boxes_of_step(k):
        out = list(static)
        for j in range(K):
            if j == k:
                continue
            out.append((P[j] if j < k else P0[j][None], sc.objects[moved[j], 4:7]))
        return out

    def held_spheres(F_ee, G, o):
        O = F_ee @ torch.linalg.inv(G)
        sp = _t(sc.obj_spheres[o])
        return apply(O, sp[None, :, :3].expand(B, -1, 3)), sp[:, 3]

    pargs = [] if want_pairs else None

    def config_collision(q, boxes, held=None):
        fr = fk_frames(r, q)
        c, rad = _robot_spheres(prob, fr)
        if held is not None:
            G, o = held
            hc, hr = held_spheres(fr[-1], G, o)
            c, rad = torch.cat([c, hc], 1), torch.cat([rad, hr])
        return _collision(c, rad, boxes, kinks, want_kinks, pargs)

    def bounds_term(v, lo, hi):
        d = dist_from_bounds(v, lo, hi)
        with torch.no_grad():
            lo_t, hi_t = _t(lo), _t(hi)
            gap = torch.minimum(v - lo_t, hi_t - v).min(-1).values
            if want_kinks:
                kinks.append(torch.minimum((v - lo_t).abs(), (v - hi_t).abs()).min(-1).values)
        return d, gap

    cols = []
    for k in range(K):
        o = moved[k]
        blk = X[:, STEP_DIM * k:STEP_DIM * (k + 1)]
        qg, qp, g = blk[:, 0:7], blk[:, 7:14], blk[:, 14:18]
        G = grasp_tf(g)
        Fg, Fp = fk_frames(r, qg), fk_frames(r, qp)
        pick_pos, pick_rot = pose_error(Fg[-1], P0[k][None] @ G)
        place_pos, place_rot = pose_error(Fp[-1], P[k] @ G)
        if want_kinks:
            with torch.no_grad():
                for e in (pick_pos, place_pos):
                    kinks.append(e.detach().clone())
                for a in (pick_rot, place_rot):
                    kinks.append(torch.minimum(a, math.pi - a).detach())
        lo_g, hi_g = prob.grasp_bounds(k)
        grasp, gap_g = bounds_term(g[:, :3], lo_g, hi_g)
        h = sc.objects[o, 4:7]
        corners = []
        for sx in (-1.0, 1.0):
            for sy in (-1.0, 1.0):
                loc = torch.tensor([[sx * h[0], sy * h[1], 0.0]], dtype=DT).expand(B, 1, 3)
                corners.append(apply(P[k], loc)[:, 0, :2])
        place = torch.zeros(B, dtype=DT)
        for cxy in corners:
            d, _ = bounds_term(cxy, sc.region_lo, sc.region_hi)
            place = place + d
        jg, gap_jg = bounds_term(qg, r.q_lo, r.q_hi)
        jp, gap_jp = bounds_term(qp, r.q_lo, r.q_hi)
        boxes = boxes_of_step(k)
        coll_g = config_collision(qg, boxes, (G, o))
        coll_p = config_collision(qp, boxes, (G, o))
        sp = _t(sc.obj_spheres[o])
        pc = apply(P[k], sp[None, :, :3].expand(B, -1, 3))
        coll_o = _collision(pc, sp[:, 3], boxes, kinks, want_kinks, pargs)
        cols += [pick_pos, pick_rot, place_pos, place_rot, grasp, place, jg, jp, coll_g, coll_p, coll_o]
        inf = torch.full((B,), math.inf, dtype=DT)
        flip_lo += [inf, inf, inf, inf, gap_g, inf, gap_jg, gap_jp, inf, inf, inf]

    W = sk.waypoints
    seg_len = []
    if W > 0:
        q0 = _t(sk.q0)[None].expand(B, 7)
        prev = q0
        for k in range(K):
            o = moved[k]
            blk = X[:, STEP_DIM * k:STEP_DIM * (k + 1)]
            qg, qp, g = blk[:, 0:7], blk[:, 7:14], blk[:, 14:18]
            G = grasp_tf(g)
            boxes = boxes_of_step(k)
            for a, b, held in ((prev, qg, None), (qg, qp, (G, o))):
                tot = torch.zeros(B, dtype=DT)
                for j in range(1, W + 1):
                    w = a + (j / (W + 1)) * (b - a)
                    tot = tot + config_collision(w, boxes, held)
                cols.append(tot)
                flip_lo.append(torch.full((B,), math.inf, dtype=DT))
                seg_len.append(torch.linalg.vector_norm(b - a, dim=-1))
                if want_kinks:
                    kinks.append(seg_len[-1].detach().clone())
            prev = qp
    if sk.self_collision:
        for k in range(K):
            blk = X[:, STEP_DIM * k:STEP_DIM * (k + 1)]
            for q in (blk[:, 0:7], blk[:, 7:14]):
                c, rad = _robot_spheres(prob, fk_frames(r, q))
                pen, top = self_collision(c, rad, r.sphere_link, kinks, want_kinks)
                cols.append(pen)
                flip_lo.append(-top)
    if sk.goal_cost:
        pos = torch.stack([P[k][:, :3, 3] for k in range(K)], 1)
        cols.append(pairwise_dist_sum(pos))
        if want_kinks:
            with torch.no_grad():
                for i in range(K):
                    for j in range(i + 1, K):
                        kinks.append(torch.linalg.vector_norm(pos[:, i] - pos[:, j], dim=-1))
    if W > 0:
        cols.append(torch.stack(seg_len, 0).sum(0))

    T = torch.stack(cols, 1)
    J = (T * _t(weights_vector(prob))).sum(1)
    return Evaluation(terms=T, cost=J, kinks=kinks, flip_lo=flip_lo, pair_args=pargs)


# ----------------------------------------------------------------------------
# batched entry points (chunked over particles; particles are independent)


def _chunks(n, size):
    for s in range(0, n, size):
        yield s, min(n, s + size)


def terms(prob: Problem, X, chunk: int = 256) -> np.ndarray:
    """[N, n_terms] unweighted term values for particle rows X [N, dim]."""
    X = torch.as_tensor(np.asarray(X, dtype=np.float64))
    out = []
    with torch.no_grad():
        for a, b in _chunks(X.shape[0], chunk):
            out.append(evaluate(prob, X[a:b]).terms)
    return torch.cat(out).numpy() if out else np.zeros((0, prob.n_terms))


def cost(prob: Problem, X, chunk: int = 256) -> np.ndarray:
    """Eq. (2): weighted sum of constraint costs and soft costs, per particle."""
    T = terms(prob, X, chunk)
    return T @ weights_vector(prob)


def mask(prob: Problem, T: np.ndarray) -> np.ndarray:
    """Eq. (3): a particle is satisfying iff every constraint term is within
    its tolerance (<=; a NaN term is never satisfied)."""
    nc = prob.n_constraint_terms
    return np.all(T[:, :nc] <= tolerance_vector(prob)[None], axis=1)


def feasibility(prob: Problem, T: np.ndarray, penalty: float):
    """Eq. (5): per constraint term c, the number of particles with
    J_c <= eps_c (NaN never), and H = mean over the constraint terms of
    h_c = that count when positive, else the penalty."""
    nc = prob.n_constraint_terms
    counts = np.sum(np.asarray(T)[:, :nc] <= tolerance_vector(prob)[None], axis=0)
    h = np.where(counts > 0, counts.astype(np.float64), float(penalty))
    return counts, float(h.mean())


def cost_and_grad(prob: Problem, X, chunk: int = 128):
    """(J [N], dJ/dx [N, dim]) by reverse-mode autodiff of the oracle's J.
    The gradient is the unscaled per-particle one; Eq. (4)'s batch mean
    multiplies it by 1/N_b."""
    X = torch.as_tensor(np.asarray(X, dtype=np.float64))
    Js, Gs = [], []
    for a, b in _chunks(X.shape[0], chunk):
        x = X[a:b].clone().requires_grad_(True)
        J = evaluate(prob, x).cost
        (g,) = torch.autograd.grad(J.sum(), x)
        Js.append(J.detach())
        Gs.append(g)
    if not Js:
        return np.zeros(0), np.zeros((0, prob.dim))
    return torch.cat(Js).numpy(), torch.cat(Gs).numpy()


def weighted_cost_and_grad(prob: Problem, X, W, chunk: int = 128):
    """Eq. (2) with per-particle weights in place of lambda: J_i = sum_c
    W[i, c] J_c(x_i), W [N, n_terms]; returns (J [N], dJ/dx [N, dim]) by
    reverse-mode autodiff of that sum."""
    X = torch.as_tensor(np.asarray(X, dtype=np.float64))
    Wt = torch.as_tensor(np.array(W, dtype=np.float64))
    Js, Gs = [], []
    for a, b in _chunks(X.shape[0], chunk):
        x = X[a:b].clone().requires_grad_(True)
        J = (evaluate(prob, x).terms * Wt[a:b]).sum(1)
        (g,) = torch.autograd.grad(J.sum(), x)
        Js.append(J.detach())
        Gs.append(g)
    if not Js:
        return np.zeros(0), np.zeros((0, prob.dim))
    return torch.cat(Js).numpy(), torch.cat(Gs).numpy()


def al_update(prob: Problem, T, mu, rho: float):
    """One method-of-multipliers step on the constraint weights: each
    constraint J_c <= eps_c is the inequality g_c = J_c - eps_c <= 0, whose
    multiplier moves to max(0, mu_c + rho g_c) (a non-finite J_c leaves it);
    the term's weight becomes lambda_c + mu_c.  Soft costs keep lambda_c and
    their multipliers.  T, mu: [N, n_terms]; returns (mu, W)."""
    T = np.asarray(T, dtype=np.float64)
    mu = np.array(mu, dtype=np.float64, copy=True)
    nc = prob.n_constraint_terms
    g = T[:, :nc] - tolerance_vector(prob)[None]
    fin = np.isfinite(T[:, :nc])
    mu[:, :nc] = np.where(fin, np.maximum(0.0, mu[:, :nc] + rho * np.where(fin, g, 0.0)), mu[:, :nc])
    W = np.broadcast_to(weights_vector(prob), T.shape).copy()
    W[:, :nc] += mu[:, :nc]
    return mu, W


def phr_weights(prob: Problem, T, mu, rho: float):
    """Gradient weights of the PHR augmented Lagrangian
    L = sum_c lambda_c J_c + (1/(2 rho)) sum_{constraints} (max(0, mu_c + rho g_c)^2 - mu_c^2),
    g_c = J_c - eps_c: W_c = lambda_c + max(0, mu_c + rho g_c) for a constraint
    (lambda_c + mu_c when J_c is not finite), lambda_c for a soft cost.
    T, mu: [N, n_terms]; returns W."""
    T = np.asarray(T, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    nc = prob.n_constraint_terms
    W = np.broadcast_to(weights_vector(prob), T.shape).copy()
    g = T[:, :nc] - tolerance_vector(prob)[None]
    fin = np.isfinite(T[:, :nc])
    W[:, :nc] += np.where(fin, np.maximum(0.0, mu[:, :nc] + rho * np.where(fin, g, 0.0)), mu[:, :nc])
    return W


def phr_lagrangian(prob: Problem, X, mu, rho: float) -> np.ndarray:
    """The PHR augmented Lagrangian itself, per particle (definition above)."""
    T = terms(prob, X)
    mu = np.asarray(mu, dtype=np.float64)
    nc = prob.n_constraint_terms
    g = T[:, :nc] - tolerance_vector(prob)[None]
    pen = (np.maximum(0.0, mu[:, :nc] + rho * g) ** 2 - mu[:, :nc] ** 2).sum(1) / (2.0 * rho)
    return T @ weights_vector(prob) + pen


def penetrating_pairs(prob: Problem, X, near: float = 1e-6):
    """Per particle: the number of sphere-box pairs with positive penetration
    max(0, r - sdf) over every collision term of Eq. (2) (robot, held-object
    and placed-object spheres of every configuration against the boxes of
    its step; waypoints included), and the number of pairs whose hinge
    argument lies within `near` of zero (where FP32 may decide otherwise)."""
    X = torch.as_tensor(np.asarray(X, dtype=np.float64))
    with torch.no_grad():
        ev = evaluate(prob, X, want_pairs=True)
    pen = sum((a > 0).sum(-1) for a in ev.pair_args)
    close = sum((a.abs() < near).sum(-1) for a in ev.pair_args)
    return pen.numpy().astype(np.int64), close.numpy().astype(np.int64)


def adam_step(x, m, v, g, t: int, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, grad_scale: float = 1.0, frozen=None, skip=None):
    """One Adam update (Kingma & Ba) of every particle coordinate, in float64.

    g is the unscaled gradient; the step uses grad_scale * g (1/N_b for the
    batch mean of Eq. (4)).  t is the 1-based update count.  Frozen
    dimensions and skipped (non-finite) particles are left untouched.
    Returns new (x, m, v).
    """
    x, m, v, g = (np.array(a, dtype=np.float64, copy=True) for a in (x, m, v, g))
    gs = grad_scale * g
    m1 = beta1 * m + (1 - beta1) * gs
    v1 = beta2 * v + (1 - beta2) * gs * gs
    m_hat = m1 / (1 - beta1 ** t)
    v_hat = v1 / (1 - beta2 ** t)
    x1 = x - lr * m_hat / (np.sqrt(v_hat) + eps)
    upd = np.ones_like(x, dtype=bool)
    if frozen is not None:
        upd &= ~np.asarray(frozen, dtype=bool)[None, :]
    if skip is not None:
        upd &= ~np.asarray(skip, dtype=bool)[:, None]
    return np.where(upd, x1, x), np.where(upd, m1, m), np.where(upd, v1, v)


def margins(prob: Problem, X, chunk: int = 256):
    """Distances that decide how FP32 may legitimately differ from FP64.

    flip [N, n_constraint]: distance of each constraint term from flipping
      its mask bit: |J_c - eps_c| when eps_c > 0; for eps_c = 0 terms, J_c
      when positive, else how deep inside its bounds the argument lies.
    kink [N]: distance to the nearest nonsmooth point of J (hinge
      arguments, interior-max ties, bound edges, zero norms, angle 0 / pi).
    """
    X = torch.as_tensor(np.asarray(X, dtype=np.float64))
    eps = tolerance_vector(prob)
    nc = prob.n_constraint_terms
    flips, kinks = [], []
    with torch.no_grad():
        for a, b in _chunks(X.shape[0], chunk):
            ev = evaluate(prob, X[a:b], want_kinks=True)
            T = ev.terms[:, :nc]
            f = torch.empty_like(T)
            for c in range(nc):
                if eps[c] > 0:
                    f[:, c] = (T[:, c] - eps[c]).abs()
                else:
                    f[:, c] = torch.where(T[:, c] > 0, T[:, c], ev.flip_lo[c].clamp(min=0.0))
            flips.append(f)
            kinks.append(torch.stack(ev.kinks, 1).min(1).values if ev.kinks
                         else torch.full((b - a,), math.inf, dtype=DT))
    return torch.cat(flips).numpy(), torch.cat(kinks).numpy()
