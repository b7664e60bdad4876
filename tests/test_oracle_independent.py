"""A second, independent formulation of every term, particle by particle, in
plain numpy + scipy: kinematics as a product of exponentials about the
zero-pose joint axes, rotations through scipy.spatial.transform, the box
distance as the distance to the point's projection onto the box (depth to the
nearest face inside), bound distances by clipping.  The batched torch oracle
must agree with it to rounding."""
import math

import numpy as np
import pytest
from scipy.spatial import distance as spd
from scipy.spatial.transform import Rotation as Rot

import oracle as O
from paper_2411_11833_amd import inputs as I


def _zero_frames(r):
    """Frames 1..7 and the tool frame at q = 0 for the alternating-twist arm."""
    d = r.dh[:, 2]
    Rm = Rot.from_rotvec([-math.pi / 2, 0, 0]).as_matrix()
    frames = []
    y = z = 0.0
    for i in range(7):
        if i % 2 == 0:
            z += d[i]
        else:
            y += d[i]
        F = np.eye(4)
        F[:3, :3] = Rm if i in (0, 2, 4) else np.eye(3)
        F[:3, 3] = (0, y, z)
        frames.append(F)
    Fe = frames[-1].copy()
    Fe[:3, 3] += (0, 0, r.tool_d)
    frames.append(Fe)
    return frames


def _poe_frames(r, q):
    d = r.dh[:, 2]
    axes = [(0, 0, 1), (0, 1, 0)] * 3 + [(0, 0, 1)]
    pts, y, z = [], 0.0, 0.0
    for i in range(7):
        pts.append(np.array([0.0, y, z]))
        if i % 2 == 0:
            z += d[i]
        else:
            y += d[i]
    zf = _zero_frames(r)
    out, T = [], np.eye(4)
    for i in range(7):
        R = Rot.from_rotvec(np.array(axes[i], float) * q[i]).as_matrix()
        E = np.eye(4)
        E[:3, :3] = R
        E[:3, 3] = (np.eye(3) - R) @ pts[i]
        T = T @ E
        out.append(T @ zf[i])
    out.append(T @ zf[7])
    return out     # index 0..6 = links 1..7, 7 = tool


def _pose(x, y, z, yaw):
    T = np.eye(4)
    T[:3, :3] = Rot.from_rotvec([0, 0, yaw]).as_matrix()
    T[:3, 3] = (x, y, z)
    return T


def _sdf(c, box_pose, h):
    p = box_pose[:3, :3].T @ (c - box_pose[:3, 3])
    if np.all(np.abs(p) <= h):
        return -np.min(h - np.abs(p))
    return np.linalg.norm(p - np.clip(p, -h, h))


def _coll(centres, radii, boxes):
    return sum(max(0.0, rr - _sdf(c, T, h)) for c, rr in zip(centres, radii) for T, h in boxes)


def _independent_terms(prob, x):
    r, sc, sk = prob.robot, prob.scene, prob.skeleton
    K = sk.n_steps
    moved = [int(o) for o in sk.object_of_step]
    ztop = sc.table[2] + sc.table[6]
    P0 = [_pose(*sc.objects[o, :4]) for o in moved]
    P = [_pose(x[21 * k + 18], x[21 * k + 19], ztop + sc.objects[moved[k], 6], x[21 * k + 20])
         for k in range(K)]
    static = [(_pose(*sc.table[:4]), sc.table[4:7])]
    static += [(_pose(*b[:4]), b[4:7]) for b in sc.obstacles]
    static += [(_pose(*sc.objects[o, :4]), sc.objects[o, 4:7])
               for o in range(len(sc.objects)) if o not in moved]

    def boxes(k):
        return static + [((P[j] if j < k else P0[j]), sc.objects[moved[j], 4:7])
                         for j in range(K) if j != k]

    def conf_coll(q, bx, G, o):
        fr = _poe_frames(r, q)
        cs = [fr[L - 1][:3, :3] @ s[:3] + fr[L - 1][:3, 3] for s, L in zip(r.spheres, r.sphere_link)]
        rad = list(r.spheres[:, 3])
        Ginv = np.linalg.inv(G)
        Obj = fr[7] @ Ginv
        for s in sc.obj_spheres[o]:
            cs.append(Obj[:3, :3] @ s[:3] + Obj[:3, 3])
            rad.append(s[3])
        return _coll(cs, rad, bx)

    def bdist(v, lo, hi):
        return np.linalg.norm(np.clip(v, lo, hi) - v)

    out = []
    for k in range(K):
        o = moved[k]
        b = x[21 * k:21 * k + 21]
        qg, qp, g = b[0:7], b[7:14], b[14:18]
        G = np.eye(4)
        G[:3, :3] = (Rot.from_rotvec([0, 0, g[3]]) * Rot.from_rotvec([math.pi, 0, 0])).as_matrix()
        G[:3, 3] = g[:3]
        Fg, Fp = _poe_frames(r, qg)[7], _poe_frames(r, qp)[7]
        row = []
        for F, Tgt in ((Fg, P0[k] @ G), (Fp, P[k] @ G)):
            row.append(np.linalg.norm(F[:3, 3] - Tgt[:3, 3]))
            row.append(Rot.from_matrix(F[:3, :3].T @ Tgt[:3, :3]).magnitude())
        lo, hi = prob.grasp_bounds(k)
        row.append(bdist(g[:3], lo, hi))
        h = sc.objects[o, 4:7]
        place = 0.0
        for sx in (-1, 1):
            for sy in (-1, 1):
                cxy = (P[k] @ np.array([sx * h[0], sy * h[1], 0.0, 1.0]))[:2]
                place += bdist(cxy, sc.region_lo, sc.region_hi)
        row.append(place)
        row.append(bdist(qg, r.q_lo, r.q_hi))
        row.append(bdist(qp, r.q_lo, r.q_hi))
        bx = boxes(k)
        row.append(conf_coll(qg, bx, G, o))
        row.append(conf_coll(qp, bx, G, o))
        pcs = [P[k][:3, :3] @ s[:3] + P[k][:3, 3] for s in sc.obj_spheres[o]]
        row.append(_coll(pcs, sc.obj_spheres[o][:, 3], bx))
        out += row
    if sk.waypoints > 0:
        W = sk.waypoints
        prev = np.asarray(sk.q0, float)
        lens = []
        for k in range(K):
            o = moved[k]
            b = x[21 * k:21 * k + 21]
            qg, qp, g = b[0:7], b[7:14], b[14:18]
            G = np.eye(4)
            G[:3, :3] = (Rot.from_rotvec([0, 0, g[3]]) * Rot.from_rotvec([math.pi, 0, 0])).as_matrix()
            G[:3, 3] = g[:3]
            bx = boxes(k)
            for a, bb, held in ((prev, qg, False), (qg, qp, True)):
                tot = 0.0
                for j in range(1, W + 1):
                    w = a + (j / (W + 1)) * (bb - a)
                    if held:
                        tot += conf_coll(w, bx, G, o)
                    else:
                        fr = _poe_frames(r, w)
                        cs = [fr[L - 1][:3, :3] @ s[:3] + fr[L - 1][:3, 3]
                              for s, L in zip(r.spheres, r.sphere_link)]
                        tot += _coll(cs, r.spheres[:, 3], bx)
                out.append(tot)
                lens.append(np.linalg.norm(bb - a))
            prev = qp
    if sk.goal_cost:
        out.append(spd.pdist(np.array([Pk[:3, 3] for Pk in P])).sum())
    if sk.waypoints > 0:
        out.append(sum(lens))
    return np.array(out)


@pytest.mark.parametrize("case", ["single", "packing", "motion"])
def test_terms_match_independent_formulation(case):
    if case == "single":
        prob = I.single_pick_place(0, 3)
    elif case == "packing":
        prob = I.packing(robot_seed=0, scene_seed=1, n_objects=3, n_obstacles=4)
    else:
        prob = I.packing(robot_seed=2, scene_seed=4, n_objects=2, n_obstacles=2, waypoints=3)
    X = I.uniform_particles(prob, 6, seed=11).astype(np.float64)
    # pull a few configurations toward the table so collisions are active
    T = O.terms(prob, X)
    for i in range(len(X)):
        want = _independent_terms(prob, X[i])
        np.testing.assert_allclose(T[i], want, rtol=1e-9, atol=1e-11)
    coll_cols = [11 * k + c for k in range(prob.skeleton.n_steps) for c in (8, 9, 10)]
    assert np.any(T[:, coll_cols] > 0)
