"""Seeded synthetic inputs: robots, box scenes, pick-place skeletons, particles.

This module only *describes* problems; it holds none of the method's
arithmetic (no kinematics, distances, costs or optimizer).  Both the CPU
oracle and the HIP path read the plain arrays produced here.

The paper's own domains, robot models and meshes are not available, so these
generators stand in for them with the shapes it describes:

* a 7-DOF revolute arm in standard Denavit-Hartenberg form (Sec. IV-B names
  forward kinematics ``FK(q)``; the experiments use 7-DOF joint positions,
  Sec. VII "Experimental Setup");
* the robot and movable objects approximated by spheres and the world by
  oriented boxes (App. "Collision Representation");
* a particle = one assignment to every continuous variable of the skeleton
  (Sec. IV-A), laid out per pick-place step as
  ``[q_grasp(7) | q_place(7) | grasp (gx, gy, gz, gyaw)(4) | place (px, py, pyaw)(3)]``;
  top-down 4-DOF grasps and 4-DOF placements (Sec. VII "Experimental Setup");
* cost weights and tolerances of App. "Cost Weights" / "Constraint Tolerances".
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Standard-DH twist pattern of an anthropomorphic 7-R arm (alternating +-90 deg).
ALPHA = (-math.pi / 2, math.pi / 2, -math.pi / 2, math.pi / 2, -math.pi / 2, math.pi / 2, 0.0)
N_JOINTS = 7
EE_LINK = 8            # sphere_link value of spheres rigid with the tool frame
STEP_DIM = 21          # per pick-place step: 7 + 7 + 4 + 3
TERMS_PER_STEP = 11
MAX_STEPS = 6

# term kinds inside one step, in storage order
TERM_NAMES = (
    "kin_pick_pos", "kin_pick_rot", "kin_place_pos", "kin_place_rot",
    "grasp", "place", "jlim_grasp", "jlim_place",
    "coll_grasp", "coll_place_conf", "coll_placed_obj",
)


@dataclass
class Robot:
    dh: np.ndarray            # [7, 4] float64: a, alpha, d, theta0 (standard DH)
    q_lo: np.ndarray          # [7]
    q_hi: np.ndarray          # [7]
    tool_d: float             # F_ee = F_7 * Tz(tool_d)
    spheres: np.ndarray       # [S, 4] x, y, z, r in the parent frame
    sphere_link: np.ndarray   # [S] int32, 1..7 = link frame, 8 = tool frame


@dataclass
class Scene:
    table: np.ndarray         # [7] cx, cy, cz, yaw, hx, hy, hz
    obstacles: np.ndarray     # [n_obs, 7]
    objects: np.ndarray       # [n_obj, 7] initial pose (cx, cy, cz, yaw) + half extents
    obj_spheres: np.ndarray   # [n_obj, n_os, 4] x, y, z, r in the object frame
    region_lo: np.ndarray     # [2] placement / goal region (x, y)
    region_hi: np.ndarray     # [2]


@dataclass
class Skeleton:
    object_of_step: np.ndarray      # [K] int32, distinct object indices, in plan order
    goal_cost: int = 0              # 1: add the pairwise placed-object distance cost
    waypoints: int = 0              # interior waypoints per transition (0 = no motion cost)
    q0: np.ndarray = field(default_factory=lambda: np.zeros(N_JOINTS))
    self_collision: int = 0         # 1: add the robot self-collision constraint at every key configuration

    @property
    def n_steps(self) -> int:
        return int(len(self.object_of_step))


@dataclass
class Weights:
    kin_pos: float = 1.0
    kin_rot: float = 5.0
    grasp: float = 1.0
    place: float = 2.0
    jlim: float = 1.0
    coll: float = 1.0
    goal: float = 0.25
    traj_len: float = 0.1
    motion_coll: float = 1.0
    self_coll: float = 1.0


@dataclass
class Tolerances:
    kin_pos: float = 0.005
    kin_rot: float = 0.05
    grasp: float = 0.0
    place: float = 0.001
    jlim: float = 0.0
    coll: float = 0.001
    motion_coll: float = 0.001
    self_coll: float = 0.0          # App. "Constraint Tolerances": zero self-penetration


@dataclass
class Problem:
    robot: Robot
    scene: Scene
    skeleton: Skeleton
    weights: Weights = field(default_factory=Weights)
    tolerances: Tolerances = field(default_factory=Tolerances)

    @property
    def dim(self) -> int:
        return STEP_DIM * self.skeleton.n_steps

    @property
    def n_motion_terms(self) -> int:
        return 2 * self.skeleton.n_steps if self.skeleton.waypoints > 0 else 0

    @property
    def n_self_terms(self) -> int:
        return 2 * self.skeleton.n_steps if self.skeleton.self_collision else 0

    @property
    def n_constraint_terms(self) -> int:
        return TERMS_PER_STEP * self.skeleton.n_steps + self.n_motion_terms + self.n_self_terms

    @property
    def n_terms(self) -> int:
        soft = (1 if self.skeleton.goal_cost else 0) + (1 if self.skeleton.waypoints > 0 else 0)
        return self.n_constraint_terms + soft

    def term_names(self) -> list[str]:
        names = [f"s{k}.{n}" for k in range(self.skeleton.n_steps) for n in TERM_NAMES]
        names += [f"motion{m}.coll" for m in range(self.n_motion_terms)]
        names += [f"self{m}" for m in range(self.n_self_terms)]
        if self.skeleton.goal_cost:
            names.append("goal")
        if self.skeleton.waypoints > 0:
            names.append("traj_len")
        return names

    def grasp_bounds(self, k: int) -> tuple[np.ndarray, np.ndarray]:
        """Valid top-down grasp positions (EE origin in the object frame):
        within the central half of the footprint, EE origin at most 2 cm
        below the top face."""
        h = self.scene.objects[self.skeleton.object_of_step[k], 4:7]
        lo = np.array([-h[0] / 2, -h[1] / 2, h[2] - 0.02])
        hi = np.array([h[0] / 2, h[1] / 2, h[2]])
        return lo, hi

    def bounds(self) -> tuple[np.ndarray, np.ndarray]:
        """Per-dimension sampling box of the uniform initializer (Sec. VII,
        the Optimization baseline initializes uniformly within bounds)."""
        lo, hi = np.zeros(self.dim), np.zeros(self.dim)
        r = self.robot
        for k in range(self.skeleton.n_steps):
            o = STEP_DIM * k
            lo[o:o + 7], hi[o:o + 7] = r.q_lo, r.q_hi
            lo[o + 7:o + 14], hi[o + 7:o + 14] = r.q_lo, r.q_hi
            glo, ghi = self.grasp_bounds(k)
            lo[o + 14:o + 17], hi[o + 14:o + 17] = glo, ghi
            lo[o + 17], hi[o + 17] = -math.pi, math.pi
            lo[o + 18:o + 20], hi[o + 18:o + 20] = self.scene.region_lo, self.scene.region_hi
            lo[o + 20], hi[o + 20] = -math.pi, math.pi
        return lo, hi


# --------------------------------------------------------------------------
# robot


def make_robot(seed: int = 0, n_spheres: int = 60, d_range=(0.1, 0.4),
               r_range=(0.03, 0.08), q_limit: float = 2.8, tool_d: float = 0.10) -> Robot:
    """Seeded 7-R arm: a_i = 0, alternating twists, link offsets d_i ~ U(d_range).

    Spheres are spread over the eight rigid segments (seven links and the
    tool) in proportion to segment length, at least one per segment.  The
    segment of link i runs from the previous frame origin, which sits at
    ``(0, -d_i sin(alpha_i), -d_i cos(alpha_i))`` in frame i, to frame i's
    origin.  Link-1 spheres stay 1 cm above the base plane and tool spheres end
    1 cm short of the tool-frame origin, so the arm never touches the table
    at its base and the gripper can reach into a grasp.
    """
    rng = np.random.default_rng(np.random.SeedSequence([0xC0B07, seed]))
    d = rng.uniform(*d_range, size=N_JOINTS)
    dh = np.zeros((N_JOINTS, 4))
    dh[:, 1] = ALPHA
    dh[:, 2] = d
    lengths = np.concatenate([d, [tool_d]])
    if n_spheres < 8:
        raise ValueError("need at least one sphere per segment")
    counts = np.ones(8, dtype=int)
    extra = n_spheres - 8
    share = lengths / lengths.sum() * extra
    counts += np.floor(share).astype(int)
    rem = n_spheres - counts.sum()
    for i in np.argsort(-(share - np.floor(share)))[:rem]:
        counts[i] += 1
    spheres, links = [], []
    for seg in range(8):
        c = counts[seg]
        radii = rng.uniform(*r_range, size=c)
        for m in range(c):
            r = radii[m]
            if seg < 7:
                al = ALPHA[seg]
                start = np.array([0.0, -d[seg] * math.sin(al), -d[seg] * math.cos(al)])
                if seg == 0:
                    s_min = (r + 0.01) / d[0]
                    s = s_min + (1.0 - s_min) * (m + 0.5) / c
                else:
                    s = (m + 0.5) / c
                p = (1.0 - s) * start
            else:
                z_top = -tool_d
                z_bot = -(r + 0.01)
                z = z_top + (z_bot - z_top) * (m + 0.5) / c if c > 1 else 0.5 * (z_top + z_bot)
                z = min(z, z_bot)
                p = np.array([0.0, 0.0, z])
            spheres.append([p[0], p[1], p[2], r])
            links.append(seg + 1)
    return Robot(dh=dh, q_lo=np.full(N_JOINTS, -q_limit), q_hi=np.full(N_JOINTS, q_limit),
                 tool_d=float(tool_d), spheres=np.array(spheres, dtype=np.float64),
                 sphere_link=np.array(links, dtype=np.int32))


# --------------------------------------------------------------------------
# scene

TABLE_CENTER = (0.3, 0.0)
TABLE_HALF = (0.5, 0.5, 0.025)


def box_spheres(half: np.ndarray, shrink: float = 0.9) -> np.ndarray:
    """Eight inset spheres at (+-hx/2, +-hy/2, +-hz/2) of radius shrink*min(h)/2:
    an under-approximation of the box, clear of its faces."""
    r = shrink * float(np.min(half)) / 2.0
    out = []
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                out.append([sx * half[0] / 2, sy * half[1] / 2, sz * half[2] / 2, r])
    return np.array(out, dtype=np.float64)


def make_scene(seed: int = 0, n_objects: int = 1, n_obstacles: int = 1,
               obj_sides=(0.04, 0.08), obs_sides=(0.03, 0.15), region_size: float = 0.3,
               region_dist=(0.35, 0.45), base_keepout: float = 0.2,
               max_tries: int = 20000) -> Scene:
    """Seeded tabletop scene: a 1 x 1 m table whose top face is z = 0, movable
    boxes and obstacle boxes resting on it at uniform yaw, and a square goal
    region at 0.35-0.45 m from the robot base.

    Footprints are kept apart (bounding circles plus 1 cm), out of the base
    keep-out disc, and out of the goal region, so that the region is free and
    every object can be picked from where it starts.
    """
    rng = np.random.default_rng(np.random.SeedSequence([0x5CE2E, seed]))
    tx, ty = TABLE_CENTER
    table = np.array([tx, ty, -TABLE_HALF[2], 0.0, *TABLE_HALF])
    x_lo, x_hi = tx - TABLE_HALF[0], tx + TABLE_HALF[0]
    y_lo, y_hi = ty - TABLE_HALF[1], ty + TABLE_HALF[1]

    for _ in range(max_tries):
        ang = rng.uniform(-math.pi, math.pi)
        dist = rng.uniform(*region_dist)
        c = np.array([dist * math.cos(ang), dist * math.sin(ang)])
        lo, hi = c - region_size / 2, c + region_size / 2
        if lo[0] >= x_lo and hi[0] <= x_hi and lo[1] >= y_lo and hi[1] <= y_hi:
            break
    else:
        raise RuntimeError("could not place goal region")
    region_lo, region_hi = lo, hi

    placed: list[tuple[float, float, float]] = []   # (x, y, radius)

    def place(half: np.ndarray) -> np.ndarray:
        rad = math.hypot(half[0], half[1])
        for _ in range(max_tries):
            x = rng.uniform(x_lo + rad, x_hi - rad)
            y = rng.uniform(y_lo + rad, y_hi - rad)
            if math.hypot(x, y) < base_keepout + rad:
                continue
            # keep clear of the goal region (grown by the footprint radius)
            if (region_lo[0] - rad - 0.01 < x < region_hi[0] + rad + 0.01 and
                    region_lo[1] - rad - 0.01 < y < region_hi[1] + rad + 0.01):
                continue
            if any(math.hypot(x - px, y - py) < rad + pr + 0.01 for px, py, pr in placed):
                continue
            placed.append((x, y, rad))
            yaw = rng.uniform(-math.pi, math.pi)
            return np.array([x, y, half[2], yaw, half[0], half[1], half[2]])
        raise RuntimeError("could not place box; scene too crowded")

    objects = np.array([place(rng.uniform(*obj_sides, size=3) / 2) for _ in range(n_objects)])
    obstacles = np.array([place(rng.uniform(*obs_sides, size=3) / 2) for _ in range(n_obstacles)])
    if n_obstacles == 0:
        obstacles = np.zeros((0, 7))
    obj_spheres = np.stack([box_spheres(o[4:7]) for o in objects]) if n_objects else np.zeros((0, 8, 4))
    return Scene(table=table, obstacles=obstacles.reshape(-1, 7), objects=objects.reshape(-1, 7),
                 obj_spheres=obj_spheres, region_lo=region_lo, region_hi=region_hi)


# --------------------------------------------------------------------------
# the standard workloads


def single_pick_place(robot_seed: int = 0, scene_seed: int = 0) -> Problem:
    """One object, one obstacle, table; one pick-place step; 40 robot spheres."""
    robot = make_robot(robot_seed, n_spheres=40)
    scene = make_scene(scene_seed, n_objects=1, n_obstacles=1)
    return Problem(robot, scene, Skeleton(object_of_step=np.array([0], dtype=np.int32)))


def packing(robot_seed: int = 0, scene_seed: int = 0, n_objects: int = 4, n_obstacles: int = 8,
            waypoints: int = 0) -> Problem:
    """Four-object packing: every object is moved into the goal region in turn,
    with the pairwise object-distance goal cost; 60 robot spheres."""
    robot = make_robot(robot_seed, n_spheres=60)
    scene = make_scene(scene_seed, n_objects=n_objects, n_obstacles=n_obstacles)
    sk = Skeleton(object_of_step=np.arange(n_objects, dtype=np.int32), goal_cost=1,
                  waypoints=waypoints)
    return Problem(robot, scene, sk)


def random_skeleton_problem(seed: int, robot: Robot, k_range=(1, 6), obs_range=(2, 12)) -> Problem:
    """A skeleton of uneven length over a scene with a random obstacle count
    (the many-skeleton batching workload)."""
    rng = np.random.default_rng(np.random.SeedSequence([0xBA7C4, seed]))
    k = int(rng.integers(k_range[0], k_range[1] + 1))
    n_obs = int(rng.integers(obs_range[0], obs_range[1] + 1))
    scene = make_scene(10_000 + seed, n_objects=k, n_obstacles=n_obs)
    sk = Skeleton(object_of_step=rng.permutation(k).astype(np.int32), goal_cost=int(k > 1))
    return Problem(robot, scene, sk)


def batch_workload(seed: int = 0, count: int = 64, robot_seed: int = 0, n_range=(512, 8192)):
    """Skeletons of uneven length (1-6 pick-place steps), each over its own
    scene with 2-12 obstacles and its own particle count, log-uniform in
    n_range and rounded to a multiple of 64.  Returns [(Problem, n)]."""
    robot = make_robot(robot_seed, n_spheres=60)
    rng = np.random.default_rng(np.random.SeedSequence([0xBA7C5, seed]))
    out = []
    for s in range(count):
        prob = random_skeleton_problem(seed * 1000 + s, robot)
        n = int(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))
        out.append((prob, max(64, (n // 64) * 64)))
    return out


# --------------------------------------------------------------------------
# particles


def uniform_particles(prob: Problem, n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Host uniform initializer: [n, dim] rows drawn in the bounds box with
    numpy's PCG64 (for parity runs; the GPU has its own counter-based one)."""
    rng = np.random.default_rng(np.random.SeedSequence([0x9A271C1E, seed]))
    lo, hi = prob.bounds()
    return (lo + (hi - lo) * rng.random((n, prob.dim))).astype(dtype)


def to_soa(x_rows: np.ndarray, ld: int | None = None, dtype=np.float32) -> np.ndarray:
    """[n, dim] rows -> dimension-major [dim, ld] buffer (columns >= n are zero)."""
    n, d = x_rows.shape
    ld = ld if ld is not None else ((n + 63) // 64) * 64
    out = np.zeros((d, ld), dtype=dtype)
    out[:, :n] = x_rows.T
    return out


# --------------------------------------------------------------------------
# seed proposer: scene features and initial network weights


def scene_features(prob: Problem, n_movable: int = 4, n_obstacles: int = 8) -> np.ndarray:
    """One row of 10 numbers per object -- centre (x, y, z), roll, pitch, yaw,
    side lengths (sx, sy, sz), movable flag -- movable objects first in the
    skeleton's order, then obstacles; missing objects are zero rows.  Boxes
    here rest flat on the table, so roll = pitch = 0."""
    rows = []
    objs = prob.scene.objects
    for k in range(n_movable):
        if k < prob.skeleton.n_steps:
            o = objs[prob.skeleton.object_of_step[k]]
            rows.append([o[0], o[1], o[2], 0.0, 0.0, o[3], 2 * o[4], 2 * o[5], 2 * o[6], 1.0])
        else:
            rows.append([0.0] * 10)
    obs = prob.scene.obstacles
    for j in range(n_obstacles):
        if j < len(obs):
            o = obs[j]
            rows.append([o[0], o[1], o[2], 0.0, 0.0, o[3], 2 * o[4], 2 * o[5], 2 * o[6], 0.0])
        else:
            rows.append([0.0] * 10)
    return np.asarray(rows, dtype=np.float64).reshape(-1)


def angle_dims(prob: Problem) -> np.ndarray:
    """1 for particle coordinates that are angles of free yaw (grasp and
    placement yaw), 0 elsewhere."""
    w = np.zeros(prob.dim, dtype=np.uint8)
    for k in range(prob.skeleton.n_steps):
        w[STEP_DIM * k + 17] = 1
        w[STEP_DIM * k + 20] = 1
    return w


def mlp_init(dims, seed: int) -> np.ndarray:
    """Flat float32 parameters (per layer W [out][in] row-major, then b) drawn
    U(-1/sqrt(in), 1/sqrt(in)), the usual default for linear layers."""
    rng = np.random.default_rng(np.random.SeedSequence([0x31F, seed]))
    parts = []
    for i, o in dims:
        a = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-a, a, i * o))
        parts.append(rng.uniform(-a, a, o))
    return np.concatenate(parts).astype(np.float32)
