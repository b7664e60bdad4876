/*
 * cutamp.h -- C ABI of the MI355X particle cost / gradient / Adam step of
 * differentiable GPU-parallelized task and motion planning (Shen et al.,
 * "Differentiable GPU-Parallelized Task and Motion Planning").
 *
 * A plan skeleton of K pick-place steps induces a continuous constraint
 * satisfaction problem (Sec. IV-A).  A *particle* is one assignment to all of
 * its continuous variables; per step k it holds 21 floats at offset 21k:
 *
 *     [ q_grasp(7) | q_place(7) | grasp gx gy gz gyaw (4) | place px py pyaw (3) ]
 *
 * Each constraint c has a cost J_c >= 0 and a tolerance eps_c; the particle
 * cost is the weighted sum of Eq. (2) and a particle is satisfying when every
 * constraint holds, Eq. (3).  A batch of N particles is optimized on the mean
 * cost of Eq. (4) with Adam (Sec. IV-B).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Particle buffers are FP32, dimension-major (structure of arrays):
 *    element (d, i) of particle i lives at X[d * ld + i], 0 <= i < n.
 *    Requirements: ld >= n, ld % 64 == 0, base pointer 256-byte aligned.
 *    The same layout and ld apply to M, V (Adam moments) and G (gradient).
 *  - All buffer arguments named X, M, V, G, cost, terms, mask, frozen and
 *    first_sat are DEVICE pointers owned by the caller.  The library never
 *    frees or keeps them, and step calls never allocate.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream); every call
 *    only enqueues work on it and returns without synchronizing.
 *  - n == 0 is a valid empty batch: the call validates and returns CT_OK
 *    without launching anything.
 *  - Return values: CT_OK, or an error code (see ct_status_string).  Argument
 *    errors are detected synchronously before any work is enqueued.  Launch
 *    failures report CT_ERR_DEVICE; faults inside a kernel surface at the
 *    caller's next synchronization.  No C++ exception crosses this boundary.
 *  - A particle with a non-finite coordinate gets a non-finite cost, mask 0,
 *    and is left untouched by Adam; this is not an error.
 *  - A problem handle is immutable after creation except for its tuning
 *    choice and graph cache; calls on one handle must not overlap in time
 *    from several host threads.  Separate handles are independent.
 */
#ifndef CUTAMP_H
#define CUTAMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CT_OK = 0,
    CT_ERR_INVALID_ARG = 1,   /* null / out-of-range / misaligned argument   */
    CT_ERR_UNSUPPORTED = 2,   /* valid request beyond the library's limits  */
    CT_ERR_ALLOC = 3,         /* device allocation failed (create only)      */
    CT_ERR_DEVICE = 4         /* a HIP runtime call or kernel launch failed  */
};

/* Limits of the library (CT_ERR_UNSUPPORTED beyond them). */
#define CT_N_JOINTS 7
#define CT_MAX_STEPS 6
#define CT_MAX_ROBOT_SPHERES 128
#define CT_MAX_STATIC_BOXES 32
#define CT_MAX_OBJECTS 24
#define CT_MAX_OBJ_SPHERES 16
#define CT_MAX_WAYPOINTS 32
#define CT_STEP_DIM 21
#define CT_TERMS_PER_STEP 11

/*
 * Robot: a 7-joint revolute arm in standard Denavit-Hartenberg form.
 * Forward kinematics FK(q) (the map named in Kin, Sec. III):
 *   F_0 = identity (base at the world origin),
 *   F_i = F_{i-1} Rz(q_i + theta0_i) Tz(d_i) Tx(a_i) Rx(alpha_i),  i = 1..7,
 *   F_ee = F_7 Tz(tool_d).
 * The robot is approximated by spheres rigid with a link frame
 * (App. "Collision Representation").
 */
typedef struct ct_robot {
    int32_t n_joints;          /* must be 7                                        */
    const double *dh;          /* [7][4]: a, alpha, d, theta0 (metres / radians)    */
    const double *q_lo;        /* [7] joint lower limits                            */
    const double *q_hi;        /* [7] joint upper limits, q_hi > q_lo               */
    double tool_d;             /* tool offset along z of frame 7                    */
    int32_t n_spheres;         /* 1 .. CT_MAX_ROBOT_SPHERES                         */
    const double *spheres;     /* [n_spheres][4]: x, y, z, radius in the parent frame; radius > 0 */
    const int32_t *sphere_link;/* [n_spheres]: 1..7 = frame F_i, 8 = tool frame F_ee */
} ct_robot;

/*
 * World: a table and obstacles as yaw-only oriented boxes, movable objects
 * (boxes approximated by spheres when moved), and a rectangular region on the
 * table that placements must lie in.  A box is 7 doubles:
 *   (cx, cy, cz, yaw, hx, hy, hz): centre, rotation about world z, half extents > 0.
 * The table's top face (cz + hz) is the support height of placements.
 */
typedef struct ct_scene {
    const double *table;       /* [7]                                               */
    int32_t n_obstacles;       /* >= 0                                               */
    const double *obstacles;   /* [n_obstacles][7]                                   */
    int32_t n_objects;         /* 1 .. CT_MAX_OBJECTS                                */
    const double *objects;     /* [n_objects][7]: initial pose (cx, cy, cz, yaw) + half extents */
    int32_t n_obj_spheres;     /* spheres per object, 1 .. CT_MAX_OBJ_SPHERES        */
    const double *obj_spheres; /* [n_objects][n_obj_spheres][4]: x, y, z, r in the object frame */
    double region_lo[2];       /* placement region (x, y), lo < hi                   */
    double region_hi[2];
} ct_scene;

/*
 * Skeleton: K pick-place steps, step k moves object object_of_step[k]
 * (Pick then Place, Listing 1).  Objects not listed stay at their initial
 * poses as obstacles.  goal_cost adds the soft pairwise distance of all
 * placed objects (the MinimizeObjDist goal action, Sec. III "Goal Costs").
 * waypoints > 0 adds, for each of the 2K transitions q0 -> q_g^1 -> q_p^1 ->
 * q_g^2 ... , a collision term over `waypoints` interior linearly
 * interpolated configurations and the soft TrajLength cost (MoveFree /
 * MoveHold, Listing 1).  self_collision = 1 adds the robot self-collision
 * constraint (Sec. IV-B "Parallelizing on GPUs"; tolerance in App.
 * "Constraint Tolerances") at each of the 2K key configurations: the sum over
 * pairs of robot spheres whose links differ by two or more (1..7 = links,
 * 8 = tool; a link and its neighbours meet at a joint and never count) of
 * max(0, r_a + r_b - |c_a - c_b|).
 */
typedef struct ct_skeleton {
    int32_t n_steps;               /* K, 1 .. CT_MAX_STEPS                          */
    const int32_t *object_of_step; /* [K] distinct indices into scene objects        */
    const double *grasp_lo;        /* [K][3] valid grasp positions (tool origin in   */
    const double *grasp_hi;        /* [K][3]  the object frame), lo <= hi            */
    int32_t goal_cost;             /* 0 or 1                                         */
    int32_t waypoints;             /* 0 .. CT_MAX_WAYPOINTS                          */
    const double *q0;              /* [7] start configuration; used if waypoints > 0 */
    int32_t self_collision;        /* 0 or 1                                         */
} ct_skeleton;

/* Weights lambda of Eq. (2) (App. "Cost Weights"). */
typedef struct ct_weights {
    double kin_pos, kin_rot, grasp, place, jlim, coll, goal, traj_len, motion_coll, self_coll;
} ct_weights;

/* Tolerances eps of Eq. (3) (App. "Constraint Tolerances"); all >= 0. */
typedef struct ct_tolerances {
    double kin_pos, kin_rot, grasp, place, jlim, coll, motion_coll, self_coll;
} ct_tolerances;

/* Adam hyper-parameters (Sec. IV-B).  grad_scale multiplies dJ/dx before the
 * moments are updated: 1/N_b gives the batch mean of Eq. (4). */
typedef struct ct_adam {
    float lr, beta1, beta2, eps, grad_scale;
} ct_adam;

typedef struct ct_problem ct_problem;

/* Human-readable name of a status code (static string, never NULL). */
const char *ct_status_string(int status);

/*
 * Validate the descriptors, build the constraint and term tables of the
 * skeleton's CSP (Sec. IV-A), and upload them to the current HIP device.
 * All descriptor pointers are host pointers, read only during the call.
 * On success *out owns the device tables (freed by ct_problem_destroy).
 * Errors: CT_ERR_INVALID_ARG, CT_ERR_UNSUPPORTED, CT_ERR_ALLOC, CT_ERR_DEVICE.
 */
int ct_problem_create(const ct_robot *robot, const ct_scene *scene, const ct_skeleton *skeleton,
                      const ct_weights *weights, const ct_tolerances *tolerances,
                      ct_problem **out);

/* Release a handle and its device tables (NULL is accepted).  Waits for the
 * device to finish (launches on any stream may still read the tables) and
 * for every replay of the handle's captured loop before releasing it. */
int ct_problem_destroy(ct_problem *problem);

/*
 * Sizes of the problem: particle dimension (21 K), number of terms, and how
 * many of them are constraints (the rest are soft costs, which never enter
 * the mask).  Term order: per step k the 11 terms
 *   kin_pick_pos, kin_pick_rot, kin_place_pos, kin_place_rot, grasp, place,
 *   jlim_grasp, jlim_place, coll_grasp, coll_place_conf, coll_placed_obj,
 * then (with waypoints) one collision term per transition, then (with
 * self_collision) one self-collision term per key configuration (q_grasp of
 * step k at 2k, q_place at 2k + 1), then the goal cost (if enabled), then
 * TrajLength (if waypoints > 0).
 * Any output pointer may be NULL.
 */
int ct_problem_info(const ct_problem *problem, int32_t *dim, int32_t *n_terms,
                    int32_t *n_constraint_terms);

/*
 * Uniform initialization within bounds (the Optimization baseline of
 * Sec. VII): joint angles in their limits, grasp positions in the grasp box,
 * yaws in [-pi, pi), placement x, y in the region.  Dimension d of particle i
 * uses Philox4x32-10 (Salmon et al., SC'11) with key (seed low, seed high
 * 32 bits) and counter (i, d / 4, 0, 0), word d % 4 -> u = (w >> 8) 2^-24,
 * x = lo_d + (hi_d - lo_d) u in FP32.  M and V, when non-NULL, are zeroed
 * for the same particles.
 */
int ct_seed_uniform(const ct_problem *problem, uint64_t seed, float *X, float *M, float *V,
                    int64_t n, int64_t ld, void *stream);

/*
 * The grasp, placement and configuration samplers of compositional particle
 * initialization (Sec. V, "Particle Initialization"): the draw of
 * ct_seed_uniform (same seed, same Philox words), except that every step's
 * placement centre is drawn uniformly over the centres that keep the
 * object's footprint, turned by the drawn placement yaw, inside the goal
 * region, so that every particle satisfies the containment of StablePlace
 * and the Grasp constraint (grasps are uniform in the valid grasp box);
 * configurations stay uniform in the joint limits (the starting points of
 * the configuration sampler, which optimizes them with grasps and
 * placements frozen).  A region narrower than the footprint on an axis
 * gives its centre on that axis.  Arguments, layout and errors as
 * ct_seed_uniform.
 */
int ct_seed_sampled(const ct_problem *problem, uint64_t seed, float *X, float *M, float *V, int64_t n,
                    int64_t ld, void *stream);

/*
 * Cost of Eq. (2) per particle: cost[i] (FP32, [n]).  Optional outputs:
 * terms [n_terms][ld] unweighted term values, and mask[i] = 1 iff particle i
 * satisfies every constraint (Eq. (3), J_c <= eps_c).  terms and mask may be
 * NULL.  X is read only.
 */
int ct_cost(const ct_problem *problem, const float *X, int64_t n, int64_t ld, float *cost,
            float *terms, uint8_t *mask, void *stream);

/*
 * Work measurement: pairs[i] = the number of (sphere, box) pairs of
 * particle i whose penetration max(0, r - sdf) is positive, over every
 * robot, held-object and placed-object sphere of every configuration and
 * the boxes of its step (the pairs whose hinge has a non-zero derivative,
 * i.e. the pairs the gradient of Eq. (2) has to visit; robot self-collision
 * pairs are not counted).  Device int32[n]; layout and errors as ct_cost.
 */
int ct_penetrating_pairs(const ct_problem *problem, const float *X, int64_t n, int64_t ld, int32_t *pairs,
                         void *stream);

/*
 * Cost and its gradient dJ/dx per particle (not scaled by 1/N_b):
 * G [dim][ld].  With weights (device [n], may be NULL) column i of G is
 * weights[i] * dJ/dx_i -- the vector-Jacobian product a reverse-mode caller
 * needs (weights = the incoming gradient of the per-particle costs).  The
 * gradient pass recomputes every configuration it needs, including the
 * motion cost's interpolated waypoints; nothing is saved between calls.
 * cost may be NULL.
 */
int ct_cost_grad(const ct_problem *problem, const float *X, int64_t n, int64_t ld, float *cost,
                 float *G, const float *weights, void *stream);

/*
 * Adam update number t (t >= 1, 1-based, bias-corrected) using the
 * gradient G: g = grad_scale * G; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * x -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 * frozen (device [dim] bytes, may be NULL) keeps dimensions fixed (the
 * paper's fixed-grasp mode).  A particle with any non-finite G or X entry is
 * left untouched.
 */
int ct_adam_apply(const ct_problem *problem, float *X, float *M, float *V, const float *G,
                  int64_t n, int64_t ld, int64_t t, const ct_adam *adam, const uint8_t *frozen,
                  void *stream);

/*
 * One fused optimization step: cost, gradient, mask and Adam update number t
 * in a single kernel (X, M, V updated in place).  cost and mask report the
 * particle *before* this update.  If some particle is satisfying,
 * *first_sat = min(*first_sat, t - 1) (an atomic on a device int the caller
 * initializes, e.g. to INT32_MAX); first_sat may be NULL.  cost and mask may
 * be NULL.
 */
int ct_step(const ct_problem *problem, float *X, float *M, float *V, int64_t n, int64_t ld,
            int64_t t, const ct_adam *adam, const uint8_t *frozen, float *cost, uint8_t *mask,
            int32_t *first_sat, void *stream);

/*
 * `iters` fused steps with updates t0+1 .. t0+iters, launched as one HIP
 * graph.  The graph is captured on first use for an argument set (t0 is not
 * part of it: the update number comes from a device counter the call sets
 * before launching) and cached in the handle; a call with other arguments
 * re-captures, which may allocate graph resources.  cost / mask hold the
 * values of the last executed step; first_sat as in ct_step.  With
 * stop_at_first != 0 (first_sat required), a step whose predecessors already
 * produced a satisfying particle does nothing, so a whole iteration budget
 * can be enqueued at once and still stops at the first solution
 * (Sec. IV-B, stopping criterion); in that mode a particle the step finds
 * satisfying is not updated, so after the stop the rows of X whose mask is 1
 * are exactly the satisfying iterates (the other rows took that step's
 * update).
 */
int ct_optimize(ct_problem *problem, float *X, float *M, float *V, int64_t n, int64_t ld,
                int64_t t0, int32_t iters, const ct_adam *adam, const uint8_t *frozen,
                float *cost, uint8_t *mask, int32_t *first_sat, int32_t stop_at_first,
                void *stream);

/*
 * Kernel shape: split = how many lanes share one particle configuration's
 * sphere list (1, 2 or 4; 0 = automatic: per call, the smallest split that
 * gives at least two workgroups per compute unit for that call's n).
 * ct_get_split reports the set value (0 = automatic).  ct_autotune times
 * every supported split on a copy of the given particles (it allocates and
 * frees scratch copies; X is not modified) and keeps the fastest; *chosen
 * (host, may be NULL) receives it.
 */
int ct_set_split(ct_problem *problem, int32_t split);
int ct_get_split(const ct_problem *problem, int32_t *split);
int ct_autotune(ct_problem *problem, const float *X, int64_t n, int64_t ld, int32_t *chosen,
                void *stream);

/*
 * Eq. (3) per pick-place step, from terms as written by ct_cost ([n_terms][ld]):
 * step_mask[k * ld_mask + i] = 1 iff every constraint term of step k of
 * particle i is within its tolerance (K rows; the motion and self-collision
 * terms belong to no step), and count[i] = the number of the particle's
 * constraint terms within tolerance (a NaN term never is).  step_mask (device
 * uint8, ld_mask >= n) and count (device int32[n]) may each be NULL.  Used to
 * pick converged actions (learned-seed training data, compositional
 * initialization).  Errors: CT_ERR_INVALID_ARG (layout as ct_cost).
 */
int ct_step_mask(const ct_problem *problem, const float *terms, int64_t n, int64_t ld, uint8_t *step_mask,
                 int64_t ld_mask, int32_t *count, void *stream);

/*
 * Plan-skeleton feasibility heuristic, Eq. (5): counts[c] = number of
 * particles i < n whose constraint term c satisfies J_c <= eps_c (terms as
 * written by ct_cost, layout [n_terms][ld]; a NaN term never counts), for
 * every constraint term c < n_constraint; H = (1/n_constraint) sum_c h_c
 * with h_c = counts[c] when positive, else `penalty` (the paper's large
 * negative Lambda_penalty, e.g. -N).  counts (device int32[n_constraint])
 * and H (device float) may each be NULL (counts then live in the handle).
 * The heuristic ranks skeletons before refinement (Sec. VI).
 */
int ct_feasibility(const ct_problem *problem, const float *terms, int64_t n, int64_t ld, float penalty,
                   int32_t *counts, float *H, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * heuristic as ct_feasibility (same kernels, identical H), with the
 * per-constraint counts kept in a static device array of CT_FEAS_SCRATCH_MAX
 * int32 per GPU instead of a caller buffer or the handle.  The call never
 * allocates or frees memory; the first call on a device looks the array's
 * address up once.  H (device float) is required; the counts stay internal.
 * Every call on one GPU shares that array, which keeps the last call's
 * counts: calls that overlap on one GPU (different streams or threads
 * without ordering) race and may return a wrong H.
 * Errors: CT_ERR_INVALID_ARG as ct_feasibility (and H == NULL);
 * CT_ERR_UNSUPPORTED when the problem has more than CT_FEAS_SCRATCH_MAX
 * constraint terms (at most 90 for the skeletons this library builds).
 */
#define CT_FEAS_SCRATCH_MAX 128
int ct_feasibility_noalloc(const ct_problem *problem, const float *terms, int64_t n, int64_t ld,
                           float penalty, float *H, void *stream);

/*
 * Augmented-Lagrangian constraint weights (Sec. IV-B names augmented
 * Lagrangians as an optimizer the method admits; Sec. "Limitations" proposes
 * them to scale the costs dynamically instead of fixing lambda).
 *
 * ct_set_term_weights makes every later ct_cost / ct_cost_grad / ct_step /
 * ct_optimize call on the handle use per-particle weights: particle i's cost
 * is sum_c W[c][i] J_c (device W [n_terms][ld], read at each launch; the
 * caller keeps it alive and may rewrite it between calls) instead of the
 * fixed lambda_c of Eq. (2).  The call's ld must equal this ld
 * (CT_ERR_INVALID_ARG otherwise).  Terms, masks and first_sat stay
 * unweighted.  W = NULL restores lambda.  A change drops the captured loop of
 * ct_optimize.  The many-skeleton calls (ct_batch_*) always use lambda.
 *
 * ct_al_update is the method-of-multipliers step between inner solves: with
 * terms [n_terms][ld] as written by ct_cost and multipliers mu [n_terms][ld]
 * (device, caller-owned, start at 0), for i < n and constraint c:
 *   mu[c][i] = max(0, mu[c][i] + rho (J_c - eps_c))   (kept if J_c is NaN/inf)
 *   W[c][i]  = lambda_c + mu[c][i]
 * and W[c][i] = lambda_c for the soft costs (their mu rows are not touched).
 * Used alone between inner solves this is dual ascent on fixed weights.
 *
 * ct_al_weights gives the weights of the PHR augmented Lagrangian
 *   L(x) = sum_c lambda_c J_c + (1 / (2 rho)) sum_c (max(0, mu_c + rho g_c)^2
 *          - mu_c^2),  g_c = J_c - eps_c  (constraints only),
 * whose gradient is sum_c W_c dJ_c/dx with
 *   W[c][i] = lambda_c + max(0, mu[c][i] + rho (J_c - eps_c))
 *   (lambda_c + mu[c][i] if J_c is NaN/inf; lambda_c for soft costs),
 * evaluated at the terms given (the particles' latest), mu unchanged.  Called
 * between short inner chunks it keeps the penalty on the current violation;
 * ct_al_update then moves the multipliers every outer step.
 * Both require rho >= 0 and finite; layouts as ct_cost.
 */
int ct_set_term_weights(ct_problem *problem, const float *W, int64_t ld);
int ct_al_update(const ct_problem *problem, const float *terms, int64_t n, int64_t ld, float rho, float *mu,
                 float *W, void *stream);
int ct_al_weights(const ct_problem *problem, const float *terms, int64_t n, int64_t ld, float rho,
                  const float *mu, float *W, void *stream);

/*
 * Compositional initialization (Sec. V): the particles of a skeleton are
 * assembled from the solutions of smaller problems, one block of rows at a
 * time.  ct_compact writes the indices i < n with mask[i] != 0, in index
 * order, to idx (device int32[n]) and their number to *count (device int32).
 * ct_gather_block sets X[row0 + r][i] = Xs[r][j] for r < rows, i < n, with
 * j = idx[i mod c] when c = *count > 0 (count may be NULL: c = 0), else
 * j = i mod n_src, and zeroes the same rows of M and V (each may be NULL).
 * Xs is [rows][lds] (lds >= n_src), X, M, V are [>= row0 + rows][ld].
 */
int ct_compact(const uint8_t *mask, int64_t n, int32_t *idx, int32_t *count, void *stream);
int ct_gather_block(const float *Xs, int64_t lds, int32_t rows, int64_t n_src, const int32_t *idx,
                    const int32_t *count, float *X, float *M, float *V, int64_t ld, int32_t row0, int64_t n,
                    void *stream);

/* ------------------------------------------------------------------------
 * Many skeletons at once (the backtracking search of Alg. 1 keeps several
 * skeletons' particle batches alive; each is optimized on its own batch mean,
 * Eq. (4)).  A batch binds problems of any lengths (K = 1..6) to their
 * caller-owned particle buffers; one optimizer iteration of every skeleton is
 * then ONE persistent kernel launch in which a fixed set of workgroups pull
 * (skeleton, particle tile) items from a device queue, largest first.
 * ------------------------------------------------------------------------ */
typedef struct ct_batch ct_batch;

/*
 * count skeletons; arrays of length count (host arrays of device pointers):
 * problems[s] (handles stay owned by the caller and must outlive the batch),
 * X/M/V[s] with layout (n[s], ld[s]) as for ct_step, cost[s] / mask[s] /
 * first_sat[s] / frozen[s] optional (the arrays themselves may be NULL).
 * Skeleton s uses grad_scale 1/n[s].  Allocates the device work tables.
 */
int ct_batch_create(int32_t count, ct_problem *const *problems, float *const *X, float *const *M,
                    float *const *V, const int64_t *n, const int64_t *ld, float *const *cost,
                    uint8_t *const *mask, int32_t *const *first_sat, const uint8_t *const *frozen,
                    ct_batch **out);
/* Release a batch (NULL is accepted); waits for the device first, like
 * ct_problem_destroy.  The problems it was built from stay valid. */
int ct_batch_destroy(ct_batch *batch);

/*
 * Launch shape: split = lanes per configuration (1, 2 or 4; 0 = default),
 * workgroups = persistent workgroups (0 = two per compute unit), persistent
 * = 0 launches one ordinary kernel per skeleton instead (the reference
 * point a persistent launch is compared with).  Rebuilds the work list.
 */
int ct_batch_set_tuning(ct_batch *batch, int32_t split, int32_t workgroups, int32_t persistent);

/* Adam update number t (>= 1) of every skeleton; lr, betas, eps from adam
 * (adam->grad_scale is ignored: each skeleton uses 1/n[s]). */
int ct_batch_step(ct_batch *batch, int64_t t, const ct_adam *adam, void *stream);

/* iters batch steps t0+1 .. t0+iters as one captured graph (cached like
 * ct_optimize's). */
int ct_batch_optimize(ct_batch *batch, int64_t t0, int32_t iters, const ct_adam *adam, void *stream);

/*
 * Times every split x {1, 2, 3, 4} workgroups per compute unit of the
 * persistent launch on the bound buffers with lr = 0 (X is not changed; M
 * and V are zeroed afterwards) and keeps the fastest.  chosen (host int[2],
 * may be NULL) receives (split, workgroups).
 */
int ct_batch_autotune(ct_batch *batch, int32_t *chosen, void *stream);

/* ------------------------------------------------------------------------
 * Learned seed proposer.  Particles are initialized by samplers before they
 * are optimized (Sec. V); this one is learned.  A multilayer perceptron maps
 * an input row [scene features (d_feat) | Gaussian noise (d_noise)] through
 * `depth` hidden layers of width `hidden` with the exact GELU x Phi(x) to
 * d_out standardized particle coordinates.  The matrix products run on the
 * matrix cores with BF16 operands (the input row, the weights, the hidden
 * activations, and in the backward pass every upstream gradient, each
 * rounded to nearest-even) and FP32 accumulation; master weights, biases,
 * gradients and Adam moments are FP32.
 *
 *  - Parameters: one flat FP32 vector, for each layer W [out][in] row-major
 *    then b [out]; ct_mlp_info gives its length.
 *  - Noise entry j of a row with counter words (c0, c1) is Box and Muller's
 *    transform of Philox4x32-10(counter = (c0, c1, j / 4, 0), key = (seed low
 *    32 bits, seed high 32 bits)): words (w0, w1) give entries 4(j/4) and
 *    4(j/4)+1, (w2, w3) the next two; u1 = 1 - (w >> 8) 2^-24, u2 = (w >> 8)
 *    2^-24, z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).
 *  - A handle owns its weights, moments, gradient and a workspace for
 *    max_rows rows (allocated in create; no other call allocates).  Calls on
 *    one handle run in stream order and must not overlap in time.
 *  - Pointers named feats, feat_of_row, draw, Y, dY, targets, params,
 *    grads, loss, chosen, mean, std, lo, hi, wrap, X, M, V are DEVICE
 *    pointers owned by the caller.  Entries of feat_of_row are clamped into
 *    [0, n_feats).
 * ------------------------------------------------------------------------ */
typedef struct ct_mlp ct_mlp;

typedef struct ct_mlp_shape {
    int32_t d_feat, d_noise; /* multiples of 4, 0 < d_feat + d_noise <= 512 */
    int32_t hidden;          /* multiple of 64, 64..4096 */
    int32_t depth;           /* hidden layers, 1..8 */
    int32_t d_out;           /* 1..512 */
    int64_t max_rows;        /* multiple of 64: most rows any call handles */
} ct_mlp_shape;

/* Allocate a handle (weights zero until ct_mlp_set_params). */
int ct_mlp_create(const ct_mlp_shape *shape, ct_mlp **out);
/* Release the handle and its buffers; waits for the device first. */
int ct_mlp_destroy(ct_mlp *mlp);
int ct_mlp_info(const ct_mlp *mlp, int64_t *n_params);

/* Copy n_params floats in (and zero the Adam moments) / out. */
int ct_mlp_set_params(ct_mlp *mlp, const float *params, void *stream);
int ct_mlp_get_params(const ct_mlp *mlp, float *params, void *stream);
/* The parameter gradient left by the last ct_mlp_backward or
 * ct_mlp_imle_step (n_params floats). */
int ct_mlp_get_grads(const ct_mlp *mlp, float *grads, void *stream);

/* FP32 noise rows out[r][d_noise] with counter words (r, draw[r]) (draw
 * NULL: (r, 0)); the generator alone, for checking. */
int ct_mlp_noise(const ct_mlp *mlp, uint64_t seed, const int32_t *draw, int64_t rows, float *out, void *stream);

/*
 * Y[r][d_out] (FP32) for rows r = 0..rows-1 (rows <= max_rows): features
 * feats[f][d_feat] with f = feat_of_row[r] (NULL: 0), noise counter words
 * (r, draw[r]) (draw NULL: (r, 0)).  Keeps the activations for
 * ct_mlp_backward.
 */
int ct_mlp_forward(ct_mlp *mlp, const float *feats, int64_t n_feats, const int32_t *feat_of_row,
                   const int32_t *draw, int64_t rows, uint64_t seed, float *Y, void *stream);
/* The same Y without keeping activations, by the kernels the nearest-draw
 * selection and seeding use (from 8,192 rows, for hidden width 512 and at
 * most 128 outputs, every layer in one launch); invalidates the
 * activations a previous ct_mlp_forward kept. */
int ct_mlp_infer(ct_mlp *mlp, const float *feats, int64_t n_feats, const int32_t *feat_of_row,
                 const int32_t *draw, int64_t rows, uint64_t seed, float *Y, void *stream);

/* Gradient of sum(dY * Y) over the last ct_mlp_forward's rows (dY
 * [rows][d_out] FP32; rows equal to that call's and a multiple of 64) into
 * the handle's gradient, overwriting it. */
int ct_mlp_backward(ct_mlp *mlp, const float *dY, int64_t rows, void *stream);

/* Adam update t (>= 1) of the parameters from grad_scale times the
 * handle's gradient; the BF16 weight copies are refreshed. */
int ct_mlp_adam(ct_mlp *mlp, int64_t t, const ct_adam *adam, void *stream);

/*
 * One implicit-maximum-likelihood training step on `rows` targets
 * (targets [rows][d_out], standardized; rows a multiple of 64, rows *
 * n_draws <= max_rows): n_draws outputs per target with noise counter
 * words (b, s); the draw whose output is nearest to the target (squared
 * Euclidean distance, each entry weighted by weights[b][d] when weights is
 * not NULL; lowest s among equals) is kept; loss = sum of the weighted
 * squared errors / (rows * d_out); backward; Adam update t.  loss (one
 * float) and chosen (int32 [rows]) may be NULL.
 */
int ct_mlp_imle_step(ct_mlp *mlp, const float *feats, int64_t n_feats, const int32_t *feat_of_row,
                     const float *targets, const float *weights, int64_t rows, int32_t n_draws, uint64_t seed, int64_t t,
                     const ct_adam *adam, float *loss, int32_t *chosen, void *stream);

/*
 * n particle seeds for one scene (features feats[d_feat]): row i uses
 * noise counter words (i, 0); x = y * std + mean, coordinates with wrap[d]
 * = 1 wrapped into [-pi, pi), every coordinate then clamped into
 * [lo[d], hi[d]]; stored as X[d * ld + i] with M and V zeroed (the particle
 * layout of ct_seed_uniform; M, V, wrap may be NULL).  mean, std, lo, hi:
 * float[d_out].  n rounded up to 64 must not exceed max_rows.
 */
int ct_mlp_sample(ct_mlp *mlp, const float *feats, uint64_t seed, const float *mean, const float *std,
                  const float *lo, const float *hi, const uint8_t *wrap, float *X, float *M, float *V, int64_t n,
                  int64_t ld, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CUTAMP_H */
