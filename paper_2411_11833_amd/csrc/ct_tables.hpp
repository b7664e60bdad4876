// Device-resident description of one skeleton's constraint problem.
//
// Built once on the host from the C-ABI descriptors and uploaded to HBM; every
// kernel reads it through a __restrict__ const pointer with wave-uniform
// indices, so the compiler serves it from the scalar cache (SGPR operands)
// rather than spending VGPRs, LDS or vector memory instructions on it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cutamp.h"

namespace ct {

// what a particle-kernel launch produces
enum Mode { MODE_COST = 0, MODE_GRAD = 1, MODE_STEP = 2 };

// lanes per workgroup of the particle kernel (four wave64s)
constexpr int WG = 256;

// A yaw-only oriented box: centre, cos/sin of its yaw, half extents.
struct Box {
    float cx, cy, cz, c, s, hx, hy, hz;
};

// A box that never moves, stored for the point-in-box-frame transform
// p = R^T (x - t) = (c x + s y + u0, c y - s x + u1, z - tz) with
// u0 = -(c tx + s ty), u1 = s tx - c ty (two FMAs per horizontal axis).
struct SBox {
    float c, s, u0, u1, tz, hx, hy, hz;
};

// weight slots
enum { W_KPOS, W_KROT, W_GRASP, W_PLACE, W_JLIM, W_COLL, W_GOAL, W_TRAJ, W_MCOLL, W_SELF, W_N };
// tolerance slots
enum { E_KPOS, E_KROT, E_GRASP, E_PLACE, E_JLIM, E_COLL, E_MCOLL, E_SELF, E_N };

// term index of each kind inside one step's block of CT_TERMS_PER_STEP
enum {
    T_PICK_POS = 0, T_PICK_ROT, T_PLACE_POS, T_PLACE_ROT, T_GRASP, T_PLACE,
    T_JLIM_G, T_JLIM_P, T_COLL_G, T_COLL_P, T_COLL_OBJ
};

struct Tables {
    int K;             // pick-place steps
    int D;             // particle dimension = 21 K
    int n_terms;       // all terms
    int n_constraint;  // terms that enter the mask
    int n_static;      // boxes that never move (table, obstacles, unmoved objects)
    int n_os;          // spheres per object
    int goal;          // pairwise placed-object distance cost on/off
    int W;             // interior waypoints per transition (0 = no motion cost)
    int goal_term;     // index of the goal term (or -1)
    int traj_term;     // index of the TrajLength term (or -1)
    int self_on;       // robot self-collision constraint at the key configurations on/off
    int self_term;     // index of the first self-collision term (slot s adds s), or -1
    int link_start[10];  // robot spheres of link L (1..8) are rs[link_start[L] .. link_start[L+1])
    float ca[CT_N_JOINTS], sa[CT_N_JOINTS], a[CT_N_JOINTS], d[CT_N_JOINTS], th0[CT_N_JOINTS];
    float q_lo[CT_N_JOINTS], q_hi[CT_N_JOINTS];
    float tool_d;
    float q0[CT_N_JOINTS];
    float w[W_N];
    float eps[E_N];
    float region_lo[2], region_hi[2];
    float4 rs[CT_MAX_ROBOT_SPHERES];           // (x, y, z, r) in the parent frame, grouped by link
    float4 lbs[10];                            // per link L: sphere (centre in the link frame, radius) holding
                                               // all of L's robot spheres, radius grown by a margin; w < 0: none
    SBox sbox[CT_MAX_STATIC_BOXES];
    Box obj0[CT_MAX_STEPS];                    // moved object of step k at its initial pose
    float p0_yaw[CT_MAX_STEPS];                // its initial yaw
    float place_z[CT_MAX_STEPS];               // centre height when placed on the table
    float grasp_lo[CT_MAX_STEPS][3], grasp_hi[CT_MAX_STEPS][3];
    float4 os[CT_MAX_STEPS][CT_MAX_OBJ_SPHERES];  // object spheres (object frame) of step k's object
    float4 obs[CT_MAX_STEPS];                  // sphere holding all of step k's object spheres (as lbs)
    float lo[CT_MAX_STEPS * CT_STEP_DIM];      // uniform-initialization box
    float hi[CT_MAX_STEPS * CT_STEP_DIM];
};

// particles per workgroup tile for a K-step skeleton and SPLIT lanes per slot
__host__ __device__ constexpr int tile_particles(int K, int SPLIT) { return WG / (2 * K * SPLIT); }

// One skeleton of a batch, as the persistent kernel sees it.
struct BatchSkel {
    const Tables* T;
    float *X, *M, *V, *cost;
    uint8_t* mask;
    int32_t* first_sat;
    const uint8_t* frozen;
    int64_t n, ld;
    float gscale;
    int pad;
};

}  // namespace ct
