// Fused particle cost / gradient / mask / Adam kernel for gfx950.
//
// What it computes (per particle x of a K-step pick-place skeleton):
//   the terms J_c of every constraint and soft cost (Sec. IV-A, App. "Cost
//   Weights"), the weighted cost J(x) of Eq. (2), the satisfaction bit of
//   Eq. (3), dJ/dx, and optionally Adam update number t on the batch-mean
//   objective of Eq. (4) (Sec. IV-B).
//
// Work decomposition (one workgroup = 256 lanes = 4 wave64s):
//   * a particle owns 2K "slots", one per robot configuration (q_grasp and
//     q_place of each step); each slot is served by SPLIT adjacent lanes that
//     share its sphere list.  A workgroup holds P = 256 / (2K SPLIT) particles;
//     lanes are slot-major, so a wave holds the same slot of many particles.
//   * phase 0 stages the particles' columns of the dimension-major X in LDS
//     (coalesced rows), phase 1 runs every lane's configuration: forward
//     kinematics, sphere transforms, sphere-vs-box penetration with its
//     adjoint fused into the same pass, pose / bound terms; gradients leave
//     the lane as world-frame wrenches folded onto the joint axes.
//   * the SPLIT lanes of a slot reduce with cross-lane shuffles; slots of a
//     particle meet in LDS; phase 2 sums each coordinate's partials in a fixed
//     order (bit-reproducible) and writes G or applies Adam in place.
//
// Box and robot-sphere tables are read with wave-uniform indices (scalar
// loads); per-lane data are the particle's own variables and the poses of
// the objects it has already placed.
#pragma once

#include "ct_tables.hpp"

namespace ct {


__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Squared distance from a point to a box, given the point in the box frame
// (p) and the half extents: ||max(|p| - h, 0)||^2, zero inside the box.
__device__ __forceinline__ float box_d2(float px, float py, float pz, float hx, float hy, float hz) {
    const float mx = fmaxf(fabsf(px) - hx, 0.f);
    const float my = fmaxf(fabsf(py) - hy, 0.f);
    const float mz = fmaxf(fabsf(pz) - hz, 0.f);
    return mx * mx + my * my + mz * mz;
}

// Penetration of a sphere that touches the box (its squared outside distance
// is below r^2), from the centre p in the box frame: pen = r - sdf with
// sdf = ||max(u, 0)|| + min(max_i u_i, 0), u = |p| - h (App. "Collision
// Representation": spheres against oriented boxes), and lam * d pen / d
// centre in world coordinates (box yaw cos c, sin s).
// Tie conventions: sign(0) = +1; among equal interior depths the lowest axis.
__device__ __forceinline__ void pair_hit(float px, float py, float pz, float r, float c, float s, float hx,
                                         float hy, float hz, float lam, float& pen, float& gx, float& gy,
                                         float& gz) {
    const float ux = fabsf(px) - hx, uy = fabsf(py) - hy, uz = fabsf(pz) - hz;
    const float mx = fmaxf(ux, 0.f), my = fmaxf(uy, 0.f), mz = fmaxf(uz, 0.f);
    const float d2 = mx * mx + my * my + mz * mz;
    float sdf, ax, ay, az;  // sdf and d sdf / d p
    if (d2 > 0.f) {
        const float inv = fast_rsq(d2);
        sdf = d2 * inv;
        ax = copysignf(mx * inv, px);
        ay = copysignf(my * inv, py);
        az = copysignf(mz * inv, pz);
    } else {
        const float sx = px >= 0.f ? 1.f : -1.f;
        const float sy = py >= 0.f ? 1.f : -1.f;
        const float sz = pz >= 0.f ? 1.f : -1.f;
        if (ux >= uy && ux >= uz) {
            sdf = ux; ax = sx; ay = 0.f; az = 0.f;
        } else if (uy >= uz) {
            sdf = uy; ax = 0.f; ay = sy; az = 0.f;
        } else {
            sdf = uz; ax = 0.f; ay = 0.f; az = sz;
        }
    }
    pen = r - sdf;
    // d pen / d centre = -R d sdf / d p
    gx = -lam * (c * ax - s * ay);
    gy = -lam * (s * ax + c * ay);
    gz = -lam * az;
}

// Poses of the moved objects as seen by one lane's step: placed by an earlier
// step (at P(rho_j), a particle variable) or still at the initial pose.
// The moved objects as seen by one lane's step k: object j (j < K) was
// placed by an earlier step (at P(rho_j), a particle variable) or is still
// at its initial pose (tables).  With the skeleton length known at compile
// time (KT > 0) the lane keeps the K poses in registers and the loops over
// them unroll; KT = 0 reads K at run time and the poses from the particle's
// staged placements in LDS (the many-skeleton kernel).
template <int KT>
struct MoveCtx {
    float x[KT], y[KT], c[KT], s[KT];
    int k;
    __device__ __forceinline__ int count() const { return KT; }
    __device__ __forceinline__ void pose(const Tables* __restrict__, int j, float& bx, float& by, float& bc,
                                         float& bs) const {
        bx = x[j]; by = y[j]; bc = c[j]; bs = s[j];
    }
};

template <>
struct MoveCtx<0> {
    const float4* plc;   // plc[j * pstride] = (x, y, cos yaw, sin yaw) of rho_j
    int pstride;
    int K, k;
    __device__ __forceinline__ int count() const { return K; }
    __device__ __forceinline__ void pose(const Tables* __restrict__ T, int j, float& bx, float& by, float& bc,
                                         float& bs) const {
        const bool placed = j < k;
        const float4 pl = plc[j * pstride];
        const Box& O = T->obj0[j];
        bx = placed ? pl.x : O.cx; by = placed ? pl.y : O.cy;
        bc = placed ? pl.z : O.c; bs = placed ? pl.w : O.s;
    }
};

// A run of NB spheres of one lane against every box of step k: static boxes
// (uniform, one scalar load per box for the whole run) and the other moved
// objects (per lane).  The NB distance tests are independent dependency
// chains; the penetration branch runs only when some lane's sphere touches
// the box.  Accumulates the unweighted penetration, each sphere's weighted
// centre gradient, and the weighted gradient with respect to the placements
// rho_j of boxes placed by earlier steps.
// Boxes that the bounding sphere (world centre w, radius rb) of some lane's
// sphere set touches: bit b of smask for static box b, bit j of omask for
// moved object j.  The masks are wave-uniform (ballot), so the sphere loops
// skip a box only when no lane of the wave needs it.  The bound holds every
// sphere of the set with a margin, so a skipped box touches none of them and
// every penetration sum is unchanged.
// The SPLIT lanes of a slot hold the same bounding sphere, so they share the
// static boxes out: lane si tests boxes si, si + SPLIT, ... (from the
// workgroup's LDS copy sbl), and the ballot bits of the lanes with a given si
// (every SPLIT-th lane of the wave) tell whether some slot touches that box.
template <int KT, int SPLIT>
__device__ __forceinline__ void touched_boxes(const Tables* __restrict__ T, const SBox* __restrict__ sbl, int si,
                                              const MoveCtx<KT>& mc, float wx, float wy, float wz, float rb,
                                              uint32_t& smask, uint32_t& omask) {
    const float r2 = rb * rb;
    smask = 0u;
    omask = 0u;
    const int nsb = T->n_static;
    constexpr uint64_t LANES = SPLIT == 1 ? ~0ull : SPLIT == 2 ? 0x5555555555555555ull : 0x1111111111111111ull;
    for (int b0 = 0; b0 < nsb; b0 += SPLIT) {
        const int b = b0 + si;
        const SBox B = sbl[min(b, nsb - 1)];
        const float px = fmaf(B.c, wx, fmaf(B.s, wy, B.u0));
        const float py = fmaf(B.c, wy, fmaf(-B.s, wx, B.u1));
        const float pz = wz - B.tz;
        const uint64_t hit = __ballot(b < nsb && box_d2(px, py, pz, B.hx, B.hy, B.hz) < r2);
#pragma unroll
        for (int u = 0; u < SPLIT; ++u)
            if (hit & (LANES << u)) smask |= 1u << (b0 + u);
    }
#pragma unroll
    for (int j = 0; j < mc.count(); ++j) {
        const Box O = T->obj0[j];
        float bx, by, bc, bs;
        mc.pose(T, j, bx, by, bc, bs);
        const float dx = wx - bx, dy = wy - by;
        const float px = bc * dx + bs * dy, py = bc * dy - bs * dx, pz = wz - O.cz;
        const bool hit = j != mc.k && box_d2(px, py, pz, O.hx, O.hy, O.hz) < r2;
        if (__ballot(hit)) omask |= 1u << j;
    }
}

template <int KT, int NB, bool GRAD>
__device__ __forceinline__ void run_vs_world(const Tables* __restrict__ T, const MoveCtx<KT>& mc, uint32_t smask,
                                             uint32_t omask, const float (&cx)[NB], const float (&cy)[NB],
                                             const float (&cz)[NB], const float (&r)[NB], float lam,
                                             float (&pen_sum)[NB], float (&gx)[NB], float (&gy)[NB],
                                             float (&gz)[NB], float* __restrict__ gr, int& nhit) {
    float r2[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) r2[m] = r[m] * r[m];
    for (uint32_t mm = smask; mm; mm &= mm - 1u) {   // the static boxes some lane's set touches
        const int b = __builtin_ctz(mm);
        const SBox B = T->sbox[b];
        bool act[NB];
        bool any = false;
        float px[NB], py[NB], pz[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            px[m] = fmaf(B.c, cx[m], fmaf(B.s, cy[m], B.u0));
            py[m] = fmaf(B.c, cy[m], fmaf(-B.s, cx[m], B.u1));
            pz[m] = cz[m] - B.tz;
            act[m] = box_d2(px[m], py[m], pz[m], B.hx, B.hy, B.hz) < r2[m];
            any |= act[m];
        }
        if (any) {
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                if (act[m]) {
                    float pen, ax, ay, az;
                    pair_hit(px[m], py[m], pz[m], r[m], B.c, B.s, B.hx, B.hy, B.hz, lam, pen, ax, ay, az);
                    pen_sum[m] += pen;
                    if (!GRAD) ++nhit;
                    if (GRAD) { gx[m] += ax; gy[m] += ay; gz[m] += az; }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < mc.count(); ++j) {   // wave-uniform trip count
        if (!((omask >> j) & 1u)) continue;   // wave-uniform
        const Box O = T->obj0[j];
        const bool placed = j < mc.k;
        float bx, by, bc, bs;
        mc.pose(T, j, bx, by, bc, bs);
        const bool on = j != mc.k;   // the step's own object is held, not an obstacle
        bool act[NB];
        bool any = false;
        float dx[NB], dy[NB], px[NB], py[NB], pz[NB];
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            dx[m] = cx[m] - bx;
            dy[m] = cy[m] - by;
            px[m] = bc * dx[m] + bs * dy[m];
            py[m] = bc * dy[m] - bs * dx[m];
            pz[m] = cz[m] - O.cz;
            act[m] = on && box_d2(px[m], py[m], pz[m], O.hx, O.hy, O.hz) < r2[m];
            any |= act[m];
        }
        if (any) {
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                if (act[m]) {
                    float pen, ax, ay, az;
                    pair_hit(px[m], py[m], pz[m], r[m], bc, bs, O.hx, O.hy, O.hz, lam, pen, ax, ay, az);
                    pen_sum[m] += pen;
                    if (!GRAD) ++nhit;
                    if (GRAD) {
                        gx[m] += ax; gy[m] += ay; gz[m] += az;
                        if (placed) {
                            // moving the box by d equals moving the sphere by -d; turning it
                            // about its own vertical axis equals turning the sphere back
                            gr[3 * j] -= ax;
                            gr[3 * j + 1] -= ay;
                            gr[3 * j + 2] -= dx[m] * ay - dy[m] * ax;
                        }
                    }
                }
            }
        }
    }
}

// Bijection from the launch index to a tile index that keeps each XCD's
// workgroups (b = x, x + 8, x + 16, ...) on a contiguous tile range.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
    constexpr int NX = 8;
    const int64_t x = b % NX, q = G / NX, rem = G % NX;
    return x * q + (x < rem ? x : rem) + b / NX;
}

// Spheres tested together against each box (independent dependency chains,
// one box load per run): 4 in the single-skeleton kernels, 2 in the
// many-skeleton kernel, whose run-time skeleton length leaves fewer registers.
template <int KT>
constexpr int run_len() { return KT > 0 ? 4 : 2; }

template <int SPLIT>
__device__ __forceinline__ float split_sum(float v) {
    if (SPLIT >= 2) v += __shfl_xor(v, 1);
    if (SPLIT >= 4) v += __shfl_xor(v, 2);
    return v;
}

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// One standard-DH joint: (R, t) <- (R, t) Rz(theta_i) Tz(d_i) Tx(a_i) Rx(alpha_i)
// for joint i (0-based) with the sine and cosine of theta_i = q_i + theta0_i.
__device__ __forceinline__ void joint_advance(const Tables* __restrict__ T, int i, float sn, float cs, float R[9],
                                              float t[3]) {
    const float ca = T->ca[i], sa = T->sa[i], a = T->a[i], d = T->d[i];
    const float lx = a * cs, ly = a * sn;
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
        const float r0 = R[3 * rr], r1 = R[3 * rr + 1], r2 = R[3 * rr + 2];
        t[rr] += r0 * lx + r1 * ly + r2 * d;
        const float w = r1 * cs - r0 * sn;
        R[3 * rr] = r0 * cs + r1 * sn;
        R[3 * rr + 1] = ca * w + r2 * sa;
        R[3 * rr + 2] = r2 * ca - sa * w;
    }
}

// NB consecutive robot spheres of one lane on a link with frame (R, t):
// lane si of a slot takes table entries s0 + si + SPLIT j, j = j0 .. j0+NB-1
// (entries past the link's end get radius 0, which never penetrates).
// Accumulates the link's wrench (force f, moment tq about the world origin).
// The sphere table is the workgroup's LDS copy (rsl), read at each lane's
// own entry.
template <int KT, int SPLIT, int NB, bool GRAD>
__device__ __forceinline__ void robot_run(const Tables* __restrict__ T, const float4* __restrict__ rsl, int s0,
                                          int s1, int j0, int si, const float R[9], const float t[3],
                                          const MoveCtx<KT>& mc, uint32_t smask, uint32_t omask, float lam,
                                          float& coll, float f[3], float tq[3], float* __restrict__ gr, int& nhit) {
    float cx[NB], cy[NB], cz[NB], rr[NB], gx[NB], gy[NB], gz[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const int e = s0 + SPLIT * (j0 + m) + si;
        const float4 sp = rsl[min(e, s1 - 1)];
        rr[m] = e < s1 ? sp.w : 0.f;
        cx[m] = R[0] * sp.x + R[1] * sp.y + R[2] * sp.z + t[0];
        cy[m] = R[3] * sp.x + R[4] * sp.y + R[5] * sp.z + t[1];
        cz[m] = R[6] * sp.x + R[7] * sp.y + R[8] * sp.z + t[2];
        gx[m] = gy[m] = gz[m] = 0.f;
    }
    // per-sphere sums over boxes, added to coll in sphere order: the same
    // additions in the same order whatever the run length
    float pen[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) pen[m] = 0.f;
    run_vs_world<KT, NB, GRAD>(T, mc, smask, omask, cx, cy, cz, rr, lam, pen, gx, gy, gz, gr, nhit);
#pragma unroll
    for (int m = 0; m < NB; ++m) coll += pen[m];
    if (GRAD) {
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            f[0] += gx[m]; f[1] += gy[m]; f[2] += gz[m];
            tq[0] += cy[m] * gz[m] - cz[m] * gy[m];
            tq[1] += cz[m] * gx[m] - cx[m] * gz[m];
            tq[2] += cx[m] * gy[m] - cy[m] * gx[m];
        }
    }
}

// All robot spheres of link L: runs of run_len, then 2, then 1, over the
// (wave-uniform) number of entries each lane of the slot handles, against the
// boxes the link's bounding sphere may touch.
template <int KT, int SPLIT, bool GRAD>
__device__ __forceinline__ void link_spheres(const Tables* __restrict__ T, const float4* __restrict__ rsl,
                                             const SBox* __restrict__ sbl, int L,
                                             int si, const float R[9], const float t[3], const MoveCtx<KT>& mc,
                                             float lam, float& coll, float f[3], float tq[3],
                                             float* __restrict__ gr, int& nhit) {
    const int s0 = T->link_start[L], s1 = T->link_start[L + 1];
    if (s1 == s0) return;
    const float4 lb = T->lbs[L];
    uint32_t smask, omask;
    touched_boxes<KT, SPLIT>(T, sbl, si, mc, R[0] * lb.x + R[1] * lb.y + R[2] * lb.z + t[0],
                      R[3] * lb.x + R[4] * lb.y + R[5] * lb.z + t[1], R[6] * lb.x + R[7] * lb.y + R[8] * lb.z + t[2],
                      lb.w, smask, omask);
    if (!(smask | omask)) return;   // wave-uniform: no sphere of the link touches any box
    const int per_lane = (s1 - s0 + SPLIT - 1) / SPLIT;
    int j = 0;
    constexpr int RUN = run_len<KT>();
    for (; j + RUN <= per_lane; j += RUN)
        robot_run<KT, SPLIT, RUN, GRAD>(T, rsl, s0, s1, j, si, R, t, mc, smask, omask, lam, coll, f, tq, gr, nhit);
    if (RUN > 2 && j + 2 <= per_lane) {
        robot_run<KT, SPLIT, 2, GRAD>(T, rsl, s0, s1, j, si, R, t, mc, smask, omask, lam, coll, f, tq, gr, nhit);
        j += 2;
    }
    for (; j < per_lane; ++j)
        robot_run<KT, SPLIT, 1, GRAD>(T, rsl, s0, s1, j, si, R, t, mc, smask, omask, lam, coll, f, tq, gr, nhit);
}

// Runs of object spheres (table osl, object frame) transformed by (R, t):
// lane si takes entries si + SPLIT j.  Returns the penetration sum; with GRAD
// accumulates the force and the moment about the world origin.
template <int KT, int SPLIT, int NB, bool GRAD>
__device__ __forceinline__ void object_run(const Tables* __restrict__ T, const float4* __restrict__ osl, int nos,
                                           int j0, int si, const float R[9], const float t[3], const MoveCtx<KT>& mc,
                                           uint32_t smask, uint32_t omask, float lam, float& coll, float f[3],
                                           float tq[3], float* __restrict__ gr, int& nhit) {
    float cx[NB], cy[NB], cz[NB], rr[NB], gx[NB], gy[NB], gz[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const int e = si + SPLIT * (j0 + m);
        const float4 sp = osl[min(e, nos - 1)];
        rr[m] = e < nos ? sp.w : 0.f;
        cx[m] = R[0] * sp.x + R[1] * sp.y + R[2] * sp.z + t[0];
        cy[m] = R[3] * sp.x + R[4] * sp.y + R[5] * sp.z + t[1];
        cz[m] = R[6] * sp.x + R[7] * sp.y + R[8] * sp.z + t[2];
        gx[m] = gy[m] = gz[m] = 0.f;
    }
    // per-sphere sums over boxes, added to coll in sphere order: the same
    // additions in the same order whatever the run length
    float pen[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) pen[m] = 0.f;
    run_vs_world<KT, NB, GRAD>(T, mc, smask, omask, cx, cy, cz, rr, lam, pen, gx, gy, gz, gr, nhit);
#pragma unroll
    for (int m = 0; m < NB; ++m) coll += pen[m];
    if (GRAD) {
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            f[0] += gx[m]; f[1] += gy[m]; f[2] += gz[m];
            tq[0] += cy[m] * gz[m] - cz[m] * gy[m];
            tq[1] += cz[m] * gx[m] - cx[m] * gz[m];
            tq[2] += cx[m] * gy[m] - cy[m] * gx[m];
        }
    }
}

template <int KT, int SPLIT, bool GRAD>
__device__ __forceinline__ void object_spheres(const Tables* __restrict__ T, const SBox* __restrict__ sbl,
                                               const float4* __restrict__ osl, int nos, float4 ob, int si, const float R[9], const float t[3],
                                               const MoveCtx<KT>& mc, float lam, float& coll, float f[3],
                                               float tq[3], float* __restrict__ gr, int& nhit) {
    if (nos <= 0) return;
    uint32_t smask, omask;
    touched_boxes<KT, SPLIT>(T, sbl, si, mc, R[0] * ob.x + R[1] * ob.y + R[2] * ob.z + t[0],
                      R[3] * ob.x + R[4] * ob.y + R[5] * ob.z + t[1], R[6] * ob.x + R[7] * ob.y + R[8] * ob.z + t[2],
                      ob.w, smask, omask);
    if (!(smask | omask)) return;   // wave-uniform: the held object touches no box
    const int per_lane = (nos + SPLIT - 1) / SPLIT;
    int j = 0;
    constexpr int RUN = run_len<KT>();
    for (; j + RUN <= per_lane; j += RUN)
        object_run<KT, SPLIT, RUN, GRAD>(T, osl, nos, j, si, R, t, mc, smask, omask, lam, coll, f, tq, gr, nhit);
    if (RUN > 2 && j + 2 <= per_lane) {
        object_run<KT, SPLIT, 2, GRAD>(T, osl, nos, j, si, R, t, mc, smask, omask, lam, coll, f, tq, gr, nhit);
        j += 2;
    }
    for (; j < per_lane; ++j)
        object_run<KT, SPLIT, 1, GRAD>(T, osl, nos, j, si, R, t, mc, smask, omask, lam, coll, f, tq, gr, nhit);
}

// dist_from_bounds of v against [lo, hi] and its gradient (scaled by lam).
template <int N>
__device__ __forceinline__ float bounds_dist(const float v[N], const float* lo, const float* hi, float lam,
                                             float g[N]) {
    float m[N], ss = 0.f;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float below = lo[j] - v[j], above = v[j] - hi[j];
        const float e = fmaxf(fmaxf(below, above), 0.f);
        m[j] = below > above ? -e : e;   // signed: d e / d v = -1 below, +1 above
        ss += e * e;
    }
    const float dist = sqrtf(ss);
    const float inv = dist > 0.f ? lam / dist : 0.f;
#pragma unroll
    for (int j = 0; j < N; ++j) g[j] = m[j] * inv;
    return dist;
}

// Robot self-collision of one configuration: pairs of robot spheres on links
// La < Lb with Lb >= La + 2, penalty max(0, r_a + r_b - |c_a - c_b|).  The
// work is done in the frame of La: the frame of every later link relative to
// it is a product of joint transforms (the stored joint sines and cosines),
// so no world frame is formed and nothing is staged.
//
// Gradient: a pair pushes its b sphere with g_b = lam (c_a - c_b) / |c_a - c_b|
// and its a sphere with -g_b along the same line, so a joint that moves both
// spheres (joints up to La) feels nothing; joint j in La+1 .. Lb (0-based
// index La .. Lb-1) feels the wrench (g_b, c_b x g_b) through its axis S_j.
// Per La, the b-side wrenches are summed by link and folded onto the axes as
// in the world pass: dJ/dq_j = <S_j, W_total> - <S_j, W of links <= j>.

// NB consecutive spheres of link Lb of one lane (entries b0 + si + SPLIT j,
// j = j0 .. j0+NB-1, in a frame (Q, o) relative to link La's frame) against
// every sphere of La (in La's own frame; uniform loads, one per NB pairs).
// Skipped when no lane's run meets La's bounding sphere (it would add zeros).
template <int SPLIT, int NB, bool GRAD>
__device__ __forceinline__ void self_run(const Tables* __restrict__ T, int a0, int a1, float4 ba, int b0, int b1,
                                         int j0, int si, const float Q[9], const float o[3], float lam, float& pen,
                                         float F[3], float Mo[3]) {
    float cx[NB], cy[NB], cz[NB], rb[NB];
    bool valid[NB];
    bool near = false;
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const int base = b0 + SPLIT * (j0 + m);   // uniform
        float4 sb = T->rs[min(base, b1 - 1)];
        if (SPLIT > 1) {
#pragma unroll
            for (int u = 1; u < SPLIT; ++u) {
                const float4 alt = T->rs[min(base + u, b1 - 1)];
                if (si == u) sb = alt;
            }
        }
        valid[m] = base + si < b1;
        rb[m] = sb.w;
        cx[m] = Q[0] * sb.x + Q[1] * sb.y + Q[2] * sb.z + o[0];
        cy[m] = Q[3] * sb.x + Q[4] * sb.y + Q[5] * sb.z + o[1];
        cz[m] = Q[6] * sb.x + Q[7] * sb.y + Q[8] * sb.z + o[2];
        const float ux = cx[m] - ba.x, uy = cy[m] - ba.y, uz = cz[m] - ba.z, ur = ba.w + sb.w;
        near |= valid[m] && ux * ux + uy * uy + uz * uz < ur * ur;
    }
    if (!__ballot(near)) return;   // wave-uniform
    float p[NB], gx[NB], gy[NB], gz[NB];
#pragma unroll
    for (int m = 0; m < NB; ++m) p[m] = gx[m] = gy[m] = gz[m] = 0.f;
    for (int a = a0; a < a1; ++a) {
        const float4 sa = T->rs[a];
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const float dx = sa.x - cx[m], dy = sa.y - cy[m], dz = sa.z - cz[m];
            const float d2 = dx * dx + dy * dy + dz * dz;
            const float rsum = sa.w + rb[m];
            if (valid[m] && d2 < rsum * rsum) {
                const float dist = sqrtf(d2);
                p[m] += rsum - dist;
                if (GRAD && dist > 0.f) {
                    const float sc = lam / dist;
                    gx[m] += dx * sc; gy[m] += dy * sc; gz[m] += dz * sc;
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        pen += p[m];
        if (GRAD) {
            F[0] += gx[m]; F[1] += gy[m]; F[2] += gz[m];
            Mo[0] += cy[m] * gz[m] - cz[m] * gy[m];
            Mo[1] += cz[m] * gx[m] - cx[m] * gz[m];
            Mo[2] += cx[m] * gy[m] - cy[m] * gx[m];
        }
    }
}

// All sphere pairs of links La and Lb (frame (Q, o) of Lb relative to La):
// runs of 2, then 1 over the entries each lane of the slot takes;
// skipped as a whole when no lane's bounding spheres of the two links meet.
template <int SPLIT, bool GRAD>
__device__ __forceinline__ void self_block(const Tables* __restrict__ T, int La, int Lb, int si, const float Q[9],
                                           const float o[3], float lam, float& pen, float F[3], float Mo[3]) {
    const int a0 = T->link_start[La], a1 = T->link_start[La + 1];
    const int b0 = T->link_start[Lb], b1 = T->link_start[Lb + 1];
    if (b0 == b1) return;
    const float4 ba = T->lbs[La], bb = T->lbs[Lb];
    const float ex = Q[0] * bb.x + Q[1] * bb.y + Q[2] * bb.z + o[0] - ba.x;
    const float ey = Q[3] * bb.x + Q[4] * bb.y + Q[5] * bb.z + o[1] - ba.y;
    const float ez = Q[6] * bb.x + Q[7] * bb.y + Q[8] * bb.z + o[2] - ba.z;
    const float rs = ba.w + bb.w;
    if (!__ballot(ex * ex + ey * ey + ez * ez < rs * rs)) return;   // wave-uniform
    const int per_lane = (b1 - b0 + SPLIT - 1) / SPLIT;
    int j = 0;
    for (; j + 2 <= per_lane; j += 2)
        self_run<SPLIT, 2, GRAD>(T, a0, a1, ba, b0, b1, j, si, Q, o, lam, pen, F, Mo);
    if (j < per_lane) self_run<SPLIT, 1, GRAD>(T, a0, a1, ba, b0, b1, j, si, Q, o, lam, pen, F, Mo);
}

// <S_j, (F, Mo)> for the axis of a frame (R, t): z . Mo + (t x z) . F
__device__ __forceinline__ float axis_dot(const float R[9], const float t[3], const float F[3], const float Mo[3]) {
    const float z[3] = {R[2], R[5], R[8]};
    float mz[3];
    cross3(t, z, mz);
    return z[0] * Mo[0] + z[1] * Mo[1] + z[2] * Mo[2] + mz[0] * F[0] + mz[1] * F[1] + mz[2] * F[2];
}

template <int SPLIT, bool GRAD>
__device__ __forceinline__ void self_pass(const Tables* __restrict__ T, int si, const float jsn[CT_N_JOINTS],
                                          const float jcs[CT_N_JOINTS], float lam, float& pen,
                                          float gq[CT_N_JOINTS]) {
#pragma unroll 1
    for (int La = 1; La <= 6; ++La) {   // wave-uniform
        if (T->link_start[La] == T->link_start[La + 1]) continue;
        float Q[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
        float o[3] = {0.f, 0.f, 0.f};
        float F[3] = {0.f, 0.f, 0.f}, Mo[3] = {0.f, 0.f, 0.f};   // b-side wrench, La's frame and origin
#pragma unroll
        for (int j = 1; j < CT_N_JOINTS; ++j) {   // (Q, o) is frame j: joint j's axis (0-based)
            if (j < La) continue;                  // wave-uniform
            if (GRAD && j > La) gq[j] -= axis_dot(Q, o, F, Mo);
            joint_advance(T, j, jsn[j], jcs[j], Q, o);
            if (j + 1 >= La + 2) self_block<SPLIT, GRAD>(T, La, j + 1, si, Q, o, lam, pen, F, Mo);
        }
        // the tool: frame 7 moved along its z-axis
        const float ot[3] = {o[0] + Q[2] * T->tool_d, o[1] + Q[5] * T->tool_d, o[2] + Q[8] * T->tool_d};
        self_block<SPLIT, GRAD>(T, La, 8, si, Q, ot, lam, pen, F, Mo);
        if (GRAD) {
            float R[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
            float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 1; j < CT_N_JOINTS; ++j) {
                if (j < La) continue;
                gq[j] += axis_dot(R, t, F, Mo);
                if (j + 1 < CT_N_JOINTS) joint_advance(T, j, jsn[j], jcs[j], R, t);
            }
        }
    }
}

// Weights of the terms one slot evaluates: the problem's lambda of Eq. (2)
// (uniform), or the particle's own row of a per-particle weight table
// [n_terms][ld] (the multiplier-adjusted weights of the augmented-Lagrangian
// mode; extended kernels only).  Fields a slot kind does not own stay unused.
struct SlotW {
    float kpos, krot, jlim, coll, mcoll, self, grasp, cobj, place, goal, traj;
};

__device__ __forceinline__ SlotW slot_weights(const Tables* __restrict__ T, const float* __restrict__ wts,
                                              int64_t ld, int64_t i, int K, int slot, bool self_on) {
    const float* w = T->w;
    SlotW sw{w[W_KPOS], w[W_KROT], w[W_JLIM], w[W_COLL], w[W_MCOLL], w[W_SELF],
             w[W_GRASP], w[W_COLL], w[W_PLACE], w[W_GOAL], w[W_TRAJ]};
    if (wts) {
        const int tb = CT_TERMS_PER_STEP * (slot >> 1);
        const bool placing = slot & 1;
        auto at = [&](int c) { return wts[(int64_t)c * ld + i]; };
        sw.kpos = at(tb + (placing ? T_PLACE_POS : T_PICK_POS));
        sw.krot = at(tb + (placing ? T_PLACE_ROT : T_PICK_ROT));
        sw.jlim = at(tb + (placing ? T_JLIM_P : T_JLIM_G));
        sw.coll = at(tb + (placing ? T_COLL_P : T_COLL_G));
        if (!placing) {
            sw.grasp = at(tb + T_GRASP);
            sw.cobj = at(tb + T_COLL_OBJ);
        } else {
            sw.place = at(tb + T_PLACE);
        }
        if (T->W > 0) {
            sw.mcoll = at(CT_TERMS_PER_STEP * K + slot);
            sw.traj = at(T->traj_term);
        }
        if (self_on) sw.self = at(T->self_term + slot);
        if (T->goal) sw.goal = at(T->goal_term);
    }
    return sw;
}

struct LaneOut {
    float cost;   // weighted sum of this slot's terms
    float traj;   // this slot's transition length (TrajLength share), 0 without motion
    int flags;    // bit 0: all of the slot's constraints hold; bit 1: finite
    int hits;     // touching sphere-box pairs of the slot (cost mode), summed over its lanes
};

// The per-configuration part of a slot's work: forward kinematics link by
// link with each link's robot spheres, the held object (optional) and the
// kinematic constraint (optional).  Accumulates the penetration sum `coll`,
// dJ/dq of this configuration into gq (folded onto the joint axes from
// world-frame wrenches: dJ/dq_j = z_j . tau + (o_j x z_j) . f for the wrench
// of everything beyond joint j), and the grasp / placement partials gg, gr.
template <int KT, int SPLIT, bool GRAD>
__device__ __forceinline__ void config_pass(const Tables* __restrict__ T, const float4* __restrict__ rsl,
                                            const SBox* __restrict__ sbl, const float4* __restrict__ osl_k, int si,
                                            const float q[CT_N_JOINTS], bool held, bool kin, bool placing,
                                            float lam, const MoveCtx<KT>& mc, float gx, float gy, float gz,
                                            float g_c, float g_s, float rho_x, float rho_y, float rho_c,
                                            float rho_s, float& coll, float gq[CT_N_JOINTS], float gg[4],
                                            float* __restrict__ gr, float& kin_pos, float& kin_rot,
                                            const SlotW* slw, bool self, float& self_pen, int& nhit) {
    const int k = mc.k;
    // Joint axis S_j = (z_j, o_j x z_j) of joint j+1 (z of frame j through its
    // origin).  dJ/dq_j = <S_j, wrench of links j+1..8>
    //                   = <S_j, total wrench> - <S_j, wrench of links 1..j>;
    // the second product (c_j) is taken on the way out, when S_j is formed
    // and links 1..j are done; the first after the tip, by a second sweep
    // over the chain that re-forms the axes from the stored joint sines and
    // cosines.  (Cancellation is bounded: an element that matters is >= 1%
    // of the largest, and the subtracted products are of that size.)
    float R[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    float t[3] = {0.f, 0.f, 0.f};
    float jsn[CT_N_JOINTS], jcs[CT_N_JOINTS], cj[CT_N_JOINTS];
    float f[3] = {0.f, 0.f, 0.f}, tq[3] = {0.f, 0.f, 0.f};   // wrench of the links done so far
#pragma unroll 1
    for (int i = 0; i < CT_N_JOINTS; ++i) {
        if (GRAD) {
            const float z[3] = {R[2], R[5], R[8]};
            float m[3];
            cross3(t, z, m);
            cj[i] = z[0] * tq[0] + z[1] * tq[1] + z[2] * tq[2] + m[0] * f[0] + m[1] * f[1] + m[2] * f[2];
        }
        float sn, cs;
        sincosf(q[i] + T->th0[i], &sn, &cs);
        jsn[i] = sn;
        jcs[i] = cs;
        joint_advance(T, i, sn, cs, R, t);
        link_spheres<KT, SPLIT, GRAD>(T, rsl, sbl, i + 1, si, R, t, mc, lam, coll, f, tq, gr, nhit);
    }
    // ---- tool frame: tool spheres, the held object, the kinematic constraint
    const float te[3] = {t[0] + R[2] * T->tool_d, t[1] + R[5] * T->tool_d, t[2] + R[8] * T->tool_d};
    link_spheres<KT, SPLIT, GRAD>(T, rsl, sbl, 8, si, R, te, mc, lam, coll, f, tq, gr, nhit);

    if (held) {
        // held object frame O = F_ee G^-1, G = Trans(g) Rz(gyaw) Rx(pi); the
        // rotation H = Rz(gyaw) Rx(pi) is symmetric and its own inverse
        const float H[9] = {g_c, g_s, 0.f, g_s, -g_c, 0.f, 0.f, 0.f, -1.f};
        float RO[9];
#pragma unroll
        for (int rr = 0; rr < 3; ++rr)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                RO[3 * rr + cc] = R[3 * rr] * H[cc] + R[3 * rr + 1] * H[3 + cc] + R[3 * rr + 2] * H[6 + cc];
        const float tO[3] = {te[0] - (RO[0] * gx + RO[1] * gy + RO[2] * gz),
                             te[1] - (RO[3] * gx + RO[4] * gy + RO[5] * gz),
                             te[2] - (RO[6] * gx + RO[7] * gy + RO[8] * gz)};
        float fo[3] = {0.f, 0.f, 0.f}, to[3] = {0.f, 0.f, 0.f};
        object_spheres<KT, SPLIT, GRAD>(T, sbl, osl_k, T->n_os, T->obs[k], si, RO, tO, mc, lam, coll, fo, to, gr,
                                        nhit);
        if (GRAD) {
            // d/dg: every held point moves by -R_O dg;  d/dgyaw: the held
            // object turns about the tool z-axis through the tool origin
            gg[0] -= RO[0] * fo[0] + RO[3] * fo[1] + RO[6] * fo[2];
            gg[1] -= RO[1] * fo[0] + RO[4] * fo[1] + RO[7] * fo[2];
            gg[2] -= RO[2] * fo[0] + RO[5] * fo[1] + RO[8] * fo[2];
            float txf[3];
            cross3(te, fo, txf);
            gg[3] += R[2] * (to[0] - txf[0]) + R[5] * (to[1] - txf[1]) + R[8] * (to[2] - txf[2]);
#pragma unroll
            for (int j = 0; j < 3; ++j) { f[j] += fo[j]; tq[j] += to[j]; }
        }
    }

    // kinematic constraint FK(q) = P G at the pick (P = initial pose) or the
    // place (P = P(rho_k)): position and rotation error
    if (kin && si == 0) {
        float Px, Py, Pz, Pc, Ps;
        if (placing) {
            Px = rho_x; Py = rho_y; Pz = T->place_z[k]; Pc = rho_c; Ps = rho_s;
        } else {
            Px = T->obj0[k].cx; Py = T->obj0[k].cy; Pz = T->obj0[k].cz; Pc = T->obj0[k].c; Ps = T->obj0[k].s;
        }
        const float Rgx = Pc * gx - Ps * gy, Rgy = Ps * gx + Pc * gy;
        const float ex = te[0] - (Px + Rgx), ey = te[1] - (Py + Rgy), ez = te[2] - (Pz + gz);
        kin_pos = sqrtf(ex * ex + ey * ey + ez * ez);
        const float cphi = Pc * g_c - Ps * g_s, sphi = Ps * g_c + Pc * g_s;
        // R_err = R_ee^T R_t with R_t columns (cphi, sphi, 0), (sphi, -cphi, 0), (0, 0, -1)
        const float E00 = R[0] * cphi + R[3] * sphi, E01 = R[0] * sphi - R[3] * cphi, E02 = -R[6];
        const float E10 = R[1] * cphi + R[4] * sphi, E11 = R[1] * sphi - R[4] * cphi, E12 = -R[7];
        const float E20 = R[2] * cphi + R[5] * sphi, E21 = R[2] * sphi - R[5] * cphi, E22 = -R[8];
        const float w0 = 0.5f * (E21 - E12), w1 = 0.5f * (E02 - E20), w2 = 0.5f * (E10 - E01);
        const float sw = sqrtf(w0 * w0 + w1 * w1 + w2 * w2);
        kin_rot = atan2f(sw, 0.5f * (E00 + E11 + E22 - 1.f));
        if (GRAD) {
            const float lp = slw ? slw->kpos : T->w[W_KPOS], lr = slw ? slw->krot : T->w[W_KROT];
            if (kin_pos > 0.f) {
                const float sc = lp / kin_pos;
                const float nx = ex * sc, ny = ey * sc, nz = ez * sc;
                f[0] += nx; f[1] += ny; f[2] += nz;
                tq[0] += te[1] * nz - te[2] * ny;
                tq[1] += te[2] * nx - te[0] * nz;
                tq[2] += te[0] * ny - te[1] * nx;
                // the target moves with the grasp offset (and the placement)
                gg[0] -= Pc * nx + Ps * ny;
                gg[1] -= -Ps * nx + Pc * ny;
                gg[2] -= nz;
                if (placing) {
                    gr[3 * k] -= nx;
                    gr[3 * k + 1] -= ny;
                    gr[3 * k + 2] -= -Rgy * nx + Rgx * ny;
                }
            }
            if (sw > 0.f) {
                const float inv = 1.f / sw;
                const float u0 = w0 * inv, u1 = w1 * inv, u2 = w2 * inv;
                const float uw0 = R[0] * u0 + R[1] * u1 + R[2] * u2;
                const float uw1 = R[3] * u0 + R[4] * u1 + R[5] * u2;
                const float uw2 = R[6] * u0 + R[7] * u1 + R[8] * u2;
                // turning the tool by w lowers the angle by u_w . w; turning the
                // target about world z raises it by u_w . z
                tq[0] -= lr * uw0; tq[1] -= lr * uw1; tq[2] -= lr * uw2;
                gg[3] += lr * uw2;
                if (placing) gr[3 * k + 2] += lr * uw2;
            }
        }
    }
    if (GRAD) {
        // second sweep: re-form each axis and take it against the total wrench
        float Q[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
        float o[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < CT_N_JOINTS; ++i) {
            const float z[3] = {Q[2], Q[5], Q[8]};
            float m[3];
            cross3(o, z, m);
            gq[i] += z[0] * tq[0] + z[1] * tq[1] + z[2] * tq[2] + m[0] * f[0] + m[1] * f[1] + m[2] * f[2] - cj[i];
            if (i + 1 < CT_N_JOINTS) joint_advance(T, i, jsn[i], jcs[i], Q, o);
        }
    }
    if (self) self_pass<SPLIT, GRAD>(T, si, jsn, jcs, slw ? slw->self : T->w[W_SELF], self_pen, gq);
}

// ---------------------------------------------------------------------------
// One slot of one particle.  Slot 2k owns q_grasp of step k and the free
// transition into it (from q_place of step k-1, or q0); slot 2k+1 owns
// q_place of step k and the holding transition q_grasp -> q_place.  Terms:
//   grasp slot: Kin at the pick, Grasp, joint limits of q_grasp, CFreeHold at
//               q_grasp, CFreePlace of the object at its placement
//   place slot: Kin at the place, StablePlace containment, joint limits of
//               q_place, CFreeHold at q_place, the goal cost (slot 1 only)
//   with waypoints: the transition's collision term over its interior
//               waypoints a + s (b - a), s = w / (W + 1), and its length.
// A waypoint's gradient goes to the transition's end (share s, this slot's
// own configuration) and start (share 1 - s, the previous slot's
// configuration, returned as the "foreign" partial).
// Every lane writes its own gradient partials (no cross-lane reduction) to
// part[0 .. 18+3K): [0,7) own q, [7,11) grasp, [11, 11+3K) placements
// (accumulated in place), [11+3K, 18+3K) foreign q.
template <int KT, int SPLIT, int MODE, bool EXT>
__device__ __forceinline__ LaneOut lane_slot(const Tables* __restrict__ T, const float* __restrict__ xs,
                                             int xs_stride, const float4* __restrict__ plc,
                                             const float4* __restrict__ osl, const float4* __restrict__ rsl,
                                             const SBox* __restrict__ sbl, int K_rt, int slot, int si,
                                             float* __restrict__ part, float* __restrict__ terms,
                                             int64_t term_ld, int64_t i_glob, bool write_terms,
                                             const float* __restrict__ wts) {
    constexpr bool GRAD = MODE != MODE_COST;
    const int K = KT ? KT : K_rt;
    const bool self_on = EXT && T->self_on;   // wave-uniform; compiled out without EXT
    // per-particle weights only in extended kernels; plain kernels read lambda
    // from the tables where each term needs it
    SlotW swv;
    if (EXT) swv = slot_weights(T, wts, term_ld, i_glob, K, slot, self_on);
    const SlotW* sw = EXT ? &swv : nullptr;
    // When a step's slots fill whole waves (the tile layout at K = 1, 2, 4)
    // the step, and at K = 1, 2 also the slot kind, is the same for every
    // lane of a wave: say so, so that step-indexed tables are scalar loads
    // and the kind's branches are uniform.
    constexpr int LANES_PER_SLOT = KT ? tile_particles(KT, SPLIT) * SPLIT : 1;
    constexpr bool STEP_UNIFORM = KT > 0 && (2 * LANES_PER_SLOT) % 64 == 0;
    constexpr bool KIND_UNIFORM = KT > 0 && LANES_PER_SLOT % 64 == 0;
    const int k = STEP_UNIFORM ? __builtin_amdgcn_readfirstlane(slot >> 1) : slot >> 1;
    const bool placing = KIND_UNIFORM ? (__builtin_amdgcn_readfirstlane(slot) & 1) : (slot & 1);
    auto X = [&](int d) { return xs[d * xs_stride]; };
    const int b0 = CT_STEP_DIM * k;
    float* gr = part + 11;   // placement partials, this lane's own

    const float gx = X(b0 + 14), gy = X(b0 + 15), gz = X(b0 + 16), gyaw = X(b0 + 17);
    float g_s, g_c;
    sincosf(gyaw, &g_s, &g_c);
    const float4 own = plc[k * xs_stride];
    const float rho_x = own.x, rho_y = own.y, rho_c = own.z, rho_s = own.w;
    MoveCtx<KT> mc;
    if constexpr (KT > 0) {
#pragma unroll
        for (int j = 0; j < KT; ++j) {
            const bool placed = j < k;
            const float4 pl = plc[j * xs_stride];
            mc.x[j] = placed ? pl.x : T->obj0[j].cx;
            mc.y[j] = placed ? pl.y : T->obj0[j].cy;
            mc.c[j] = placed ? pl.z : T->obj0[j].c;
            mc.s[j] = placed ? pl.w : T->obj0[j].s;
        }
        mc.k = k;
    } else {
        mc = MoveCtx<0>{plc, xs_stride, K, k};
    }
    if (GRAD) {
        for (int j = 0; j < 3 * K; ++j) gr[j] = 0.f;
    }

    // this slot's configuration (the transition's end b, row qb_row of the
    // staged particle) and the transition's start a (row qa_row, or q0)
    const int W = T->W;
    const int qb_row = b0 + (placing ? 7 : 0);
    const bool start_is_var = placing || k > 0;
    const int qa_row = placing ? b0 : b0 - CT_STEP_DIM + 7;
    auto qb = [&](int j) { return X(qb_row + j); };
    auto qa = [&](int j) { return start_is_var ? X(qa_row + j) : T->q0[j]; };

    float gq[CT_N_JOINTS], gqa[CT_N_JOINTS];
#pragma unroll
    for (int j = 0; j < CT_N_JOINTS; ++j) gq[j] = gqa[j] = 0.f;
    float gg[4] = {0.f, 0.f, 0.f, 0.f};
    float coll = 0.f, coll_m = 0.f, kin_pos = 0.f, kin_rot = 0.f, selfc = 0.f;
    int nhit = 0;   // touching sphere-box pairs (cost mode only; the adjoint's work)
    const float4* osl_k = osl + k * CT_MAX_OBJ_SPHERES;

    // waypoints w = 1..W of the transition, then the configuration itself
    for (int w = 1; w <= W + 1; ++w) {
        const bool key = w == W + 1;   // wave-uniform
        const float s = key ? 1.f : (float)w / (float)(W + 1);
        float q[CT_N_JOINTS], gw[CT_N_JOINTS];
#pragma unroll
        for (int j = 0; j < CT_N_JOINTS; ++j) {
            const float b = qb(j);
            q[j] = key ? b : qa(j) + s * (b - qa(j));
            gw[j] = 0.f;
        }
        float cw = 0.f;
        // the object is in the hand at both configurations of its step and
        // along the holding transition
        const bool held = key || placing;
        const float lam = key ? (sw ? sw->coll : T->w[W_COLL]) : (sw ? sw->mcoll : T->w[W_MCOLL]);
        config_pass<KT, SPLIT, GRAD>(T, rsl, sbl, osl_k, si, q, held, key, placing, lam, mc, gx, gy, gz, g_c, g_s, rho_x, rho_y,
                                     rho_c, rho_s, cw, gw, gg, gr, kin_pos, kin_rot, sw, key && self_on, selfc, nhit);
        if (key) coll += cw; else coll_m += cw;
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < CT_N_JOINTS; ++j) {
                gq[j] += s * gw[j];
                gqa[j] += (1.f - s) * gw[j];
            }
        }
    }
    if (!start_is_var) {
#pragma unroll
        for (int j = 0; j < CT_N_JOINTS; ++j) gqa[j] = 0.f;
    }

    // joint limits of this configuration; the transition's length
    float jlim = 0.f, traj = 0.f;
    if (si == 0) {
        float gj[CT_N_JOINTS], qk[CT_N_JOINTS];
#pragma unroll
        for (int j = 0; j < CT_N_JOINTS; ++j) qk[j] = qb(j);
        jlim = bounds_dist<CT_N_JOINTS>(qk, T->q_lo, T->q_hi, sw ? sw->jlim : T->w[W_JLIM], gj);
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < CT_N_JOINTS; ++j) gq[j] += gj[j];
        }
        if (W > 0) {
            float ss = 0.f;
#pragma unroll
            for (int j = 0; j < CT_N_JOINTS; ++j) ss += (qb(j) - qa(j)) * (qb(j) - qa(j));
            traj = sqrtf(ss);
            if (GRAD && traj > 0.f) {
                const float sc = (sw ? sw->traj : T->w[W_TRAJ]) / traj;
#pragma unroll
                for (int j = 0; j < CT_N_JOINTS; ++j) {
                    gq[j] += sc * (qb(j) - qa(j));
                    if (start_is_var) gqa[j] -= sc * (qb(j) - qa(j));
                }
            }
        }
    }

    float grasp = 0.f, coll_obj = 0.f, place = 0.f, goal = 0.f;
    const float lc = sw ? sw->cobj : T->w[W_COLL];
    if (!placing) {
        if (si == 0) {
            const float gv[3] = {gx, gy, gz};
            float gb[3];
            grasp = bounds_dist<3>(gv, T->grasp_lo[k], T->grasp_hi[k], sw ? sw->grasp : T->w[W_GRASP], gb);
            if (GRAD) { gg[0] += gb[0]; gg[1] += gb[1]; gg[2] += gb[2]; }
        }
        // CFreePlace: the object's spheres at its placement P(rho_k); the
        // object frame's force and moment give the placement gradient
        const float Rp[9] = {rho_c, -rho_s, 0.f, rho_s, rho_c, 0.f, 0.f, 0.f, 1.f};
        const float tp[3] = {rho_x, rho_y, T->place_z[k]};
        float fp[3] = {0.f, 0.f, 0.f}, mp[3] = {0.f, 0.f, 0.f};
        object_spheres<KT, SPLIT, GRAD>(T, sbl, osl_k, T->n_os, T->obs[k], si, Rp, tp, mc, lc, coll_obj, fp, mp, gr,
                                        nhit);
        if (GRAD) {
            // translation: the force; turning about the vertical through the
            // placement origin: z of the moment about that point
            gr[3 * k] += fp[0];
            gr[3 * k + 1] += fp[1];
            gr[3 * k + 2] += mp[2] - (tp[0] * fp[1] - tp[1] * fp[0]);
        }
    } else if (si == 0) {
        // StablePlace containment: footprint corners inside the region
        const float hx = T->obj0[k].hx, hy = T->obj0[k].hy, lpl = sw ? sw->place : T->w[W_PLACE];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const float sx = (cc & 1) ? hx : -hx, sy = (cc & 2) ? hy : -hy;
            const float vx = rho_c * sx - rho_s * sy, vy = rho_s * sx + rho_c * sy;
            const float cv[2] = {rho_x + vx, rho_y + vy};
            float gcr[2];
            place += bounds_dist<2>(cv, T->region_lo, T->region_hi, lpl, gcr);
            if (GRAD) {
                gr[3 * k] += gcr[0];
                gr[3 * k + 1] += gcr[1];
                gr[3 * k + 2] += -vy * gcr[0] + vx * gcr[1];
            }
        }
        if (slot == 1 && T->goal) {
            // MinimizeObjDist: sum of pairwise distances of the placements
            const float lg = sw ? sw->goal : T->w[W_GOAL];
            for (int a = 0; a < K; ++a)
                for (int b = a + 1; b < K; ++b) {
                    const float dx = plc[a * xs_stride].x - plc[b * xs_stride].x;
                    const float dy = plc[a * xs_stride].y - plc[b * xs_stride].y;
                    const float dz = T->place_z[a] - T->place_z[b];
                    const float dist = sqrtf(dx * dx + dy * dy + dz * dz);
                    goal += dist;
                    if (GRAD && dist > 0.f) {
                        const float sc = lg / dist;
                        gr[3 * a] += dx * sc; gr[3 * a + 1] += dy * sc;
                        gr[3 * b] -= dx * sc; gr[3 * b + 1] -= dy * sc;
                    }
                }
        }
    }

    // ---- penetration sums of the slot (all SPLIT lanes contribute)
    coll = split_sum<SPLIT>(coll);
    coll_m = split_sum<SPLIT>(coll_m);
    coll_obj = split_sum<SPLIT>(coll_obj);
    if (self_on) selfc = split_sum<SPLIT>(selfc);

    LaneOut out;
    const float* e = T->eps;
    float gsum = 0.f;
    if (GRAD) {
#pragma unroll
        for (int j = 0; j < CT_N_JOINTS; ++j) {
            part[j] = gq[j];
            part[11 + 3 * K + j] = gqa[j];
            gsum += gq[j] + gqa[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) { part[7 + j] = gg[j]; gsum += gg[j]; }
        for (int j = 0; j < 3 * K; ++j) gsum += gr[j];
    }
    const SlotW swc = sw ? *sw : SlotW{T->w[W_KPOS], T->w[W_KROT], T->w[W_JLIM], T->w[W_COLL], T->w[W_MCOLL],
                                       T->w[W_SELF], T->w[W_GRASP], T->w[W_COLL], T->w[W_PLACE], T->w[W_GOAL],
                                       T->w[W_TRAJ]};
    float kw = swc.kpos * kin_pos + swc.krot * kin_rot + swc.jlim * jlim + swc.coll * coll + swc.mcoll * coll_m +
               swc.traj * traj;
    bool ok = kin_pos <= e[E_KPOS] && kin_rot <= e[E_KROT] && jlim <= e[E_JLIM] && coll <= e[E_COLL] &&
              coll_m <= e[E_MCOLL];
    if (self_on) {
        kw += swc.self * selfc;
        ok = ok && selfc <= e[E_SELF];
    }
    if (!placing) {
        out.cost = kw + swc.grasp * grasp + swc.cobj * coll_obj;
        ok = ok && grasp <= e[E_GRASP] && coll_obj <= e[E_COLL];
    } else {
        out.cost = kw + swc.place * place + swc.goal * goal;
        ok = ok && place <= e[E_PLACE];
    }
    out.traj = traj;
    out.hits = 0;
    if (!GRAD) out.hits = (int)split_sum<SPLIT>((float)nhit);   // exact: small integers
    // a slot is finite when its own cost and every lane's partials are
    const float gtot = split_sum<SPLIT>(gsum);
    const bool fin = __builtin_isfinite(out.cost) && __builtin_isfinite(gtot);
    out.flags = (ok ? 1 : 0) | (fin ? 2 : 0);

    if (write_terms && si == 0) {
        const int tb = CT_TERMS_PER_STEP * k;
        auto put = [&](int idx, float v) { terms[(int64_t)idx * term_ld + i_glob] = v; };
        if (!placing) {
            put(tb + T_PICK_POS, kin_pos);
            put(tb + T_PICK_ROT, kin_rot);
            put(tb + T_GRASP, grasp);
            put(tb + T_JLIM_G, jlim);
            put(tb + T_COLL_G, coll);
            put(tb + T_COLL_OBJ, coll_obj);
        } else {
            put(tb + T_PLACE_POS, kin_pos);
            put(tb + T_PLACE_ROT, kin_rot);
            put(tb + T_PLACE, place);
            put(tb + T_JLIM_P, jlim);
            put(tb + T_COLL_P, coll);
            if (slot == 1 && T->goal) put(T->goal_term, goal);
        }
        if (W > 0) put(CT_TERMS_PER_STEP * K + slot, coll_m);
        if (self_on) put(T->self_term + slot, selfc);
    }
    return out;
}

// ---------------------------------------------------------------------------
// Workgroup-level tile: P particles x 2K slots x SPLIT lanes, K at run time.

// Largest LDS footprint over K = 1..CT_MAX_STEPS for a given SPLIT:
//   staged particles  D P = 21 K floor(128 / (K SPLIT))  <= 2688 / SPLIT floats
//   placements        K P                                <= 128 / SPLIT float4
//   lane partials     P 2K SPLIT (18 + 3K)                <= 256 (18 + 3 * 6) floats
//   slot records      P 2K                                <= 256 / SPLIT
//   staged moments    2 D P (fused step only; the same bound as the particles)
template <int SPLIT>
struct TileSmem {
    float xs[2688 / SPLIT];
    float ms[2688 / SPLIT], vs[2688 / SPLIT];
    uint8_t frz[CT_MAX_STEPS * CT_STEP_DIM];
    float4 rs[CT_MAX_ROBOT_SPHERES];
    SBox sbx[CT_MAX_STATIC_BOXES];
    float4 plc[128 / SPLIT];
    float part[WG * (18 + 3 * CT_MAX_STEPS)];
    float cpart[WG / SPLIT];
    float tpart[WG / SPLIT];
    int flg[WG / SPLIT];
    int hpart[WG / SPLIT];
    int okp[128 / SPLIT];
    float4 osl[CT_MAX_STEPS * CT_MAX_OBJ_SPHERES];
    int any_sat;
};

// What one tile reads and writes (one skeleton's buffers).
struct TileIO {
    const Tables* T;
    float *X, *M, *V, *G, *cost, *terms;
    uint8_t* mask;
    int32_t* first_sat;
    const uint8_t* frozen;
    const float* gw;
    int64_t n, ld;
    float gscale;
    const float* wts;   // per-particle term weights [n_terms][ld] (extended kernels), or null
    int keep_sat = 0;   // stop-at-first: a satisfying particle is not updated, so X keeps it
    int32_t* hits = nullptr;   // cost mode: touching sphere-box pairs per particle, or null
};


template <int KT, int SPLIT, int MODE, bool EXT>
__device__ __forceinline__ void run_tile(const TileIO& io, int64_t p0, TileSmem<SPLIT>& sm, float lr, float b1,
                                         float b2, float eps, int32_t t) {
    const Tables* __restrict__ T = io.T;
    const int K = KT ? KT : T->K;
    const int SLOTS = 2 * K;
    const int LPP = SLOTS * SPLIT;
    const int P = WG / LPP;
    const int D = CT_STEP_DIM * K;
    const int NP = 18 + 3 * K;
    const int64_t n = io.n, ld = io.ld;
    const int tid = threadIdx.x;
    const int32_t iter = t - 1;

    // phase 0: stage this tile's particles (coalesced along particles) and,
    // for the fused step, their Adam moments and the frozen flags; the
    // placements' poses, and the robot and object sphere tables.  A lane
    // issues all of its loads before the first wait (NST is an upper bound
    // on its share; with the skeleton length known at compile time, exact),
    // so the tile pays one memory latency here and none in phase 2.
    {
        constexpr int NST = (KT ? CT_STEP_DIM * KT * tile_particles(KT, SPLIT) : 2688 / SPLIT) / WG + 1;
        constexpr bool MV = MODE == MODE_STEP;
        float xv[NST], mv[NST], vv[NST];
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = tid + u * WG;
            const int d = idx / P, p = idx - d * P;
            const int64_t i = p0 + p;
            xv[u] = mv[u] = vv[u] = 0.f;
            if (idx < D * P && i < n) {
                const int64_t a = d * ld + i;
                xv[u] = io.X[a];
                if (MV) { mv[u] = io.M[a]; vv[u] = io.V[a]; }
            }
        }
        if (MV && tid < D) sm.frz[tid] = io.frozen ? io.frozen[tid] : 0;
#pragma unroll
        for (int u = 0; u < NST; ++u) {
            const int idx = tid + u * WG;
            if (idx < D * P) {
                sm.xs[idx] = xv[u];
                if (MV) { sm.ms[idx] = mv[u]; sm.vs[idx] = vv[u]; }
            }
        }
    }
    for (int idx = tid; idx < K * CT_MAX_OBJ_SPHERES; idx += WG)
        sm.osl[idx] = T->os[idx / CT_MAX_OBJ_SPHERES][idx % CT_MAX_OBJ_SPHERES];
    for (int idx = tid; idx < T->link_start[9]; idx += WG) sm.rs[idx] = T->rs[idx];
    if (tid < T->n_static) sm.sbx[tid] = T->sbox[tid];
    if (tid == 0) sm.any_sat = 0;
    __syncthreads();
    for (int idx = tid; idx < K * P; idx += WG) {
        const int j = idx / P, p = idx - j * P;
        const float* col = sm.xs + p;
        float sj, cj;
        sincosf(col[(CT_STEP_DIM * j + 20) * P], &sj, &cj);
        sm.plc[idx] = make_float4(col[(CT_STEP_DIM * j + 18) * P], col[(CT_STEP_DIM * j + 19) * P], cj, sj);
    }
    __syncthreads();

    // phase 1: every lane evaluates its slot.  Lanes are slot-major (the SPLIT
    // lanes of a slot adjacent, then the tile's particles, then the slots), so
    // a wave serves one or two slots of many particles: the same step and kind
    // of configuration, hence uniform branches and coherent box masks.
    {
        const int si = tid % SPLIT, rest = tid / SPLIT;
        const int slot = rest / P, p = rest - slot * P;
        if (slot < SLOTS) {
            const int64_t i = p0 + p;
            const bool wt = (MODE == MODE_COST) && io.terms != nullptr && i < n;
            const LaneOut o = lane_slot<KT, SPLIT, MODE, EXT>(T, sm.xs + p, P, sm.plc + p, sm.osl, sm.rs, sm.sbx, K, slot, si,
                                                     sm.part + (size_t)((p * SLOTS + slot) * SPLIT + si) * NP,
                                                     io.terms, ld, i, wt, i < n ? io.wts : nullptr);
            if (si == 0) {
                sm.cpart[p * SLOTS + slot] = o.cost;
                sm.tpart[p * SLOTS + slot] = o.traj;
                sm.flg[p * SLOTS + slot] = o.flags;
                if (MODE == MODE_COST) sm.hpart[p * SLOTS + slot] = o.hits;
            }
        }
    }
    __syncthreads();

    // phase 1.5: per-particle cost, mask, update permission
    if (tid < P) {
        const int64_t i = p0 + tid;
        float J = 0.f;
        int m = 1, ok = 1;
        for (int s = 0; s < SLOTS; ++s) {
            J += sm.cpart[tid * SLOTS + s];
            m &= sm.flg[tid * SLOTS + s] & 1;
            ok &= (sm.flg[tid * SLOTS + s] >> 1) & 1;
        }
        ok &= __builtin_isfinite(J) ? 1 : 0;
        m &= __builtin_isfinite(J) ? 1 : 0;
        // the solution returned on stop is the satisfying iterate itself
        // (the pre-update x the mask describes), so it keeps its value
        sm.okp[tid] = ok & (io.keep_sat ? 1 - m : 1);
        if (i < n) {
            if (MODE == MODE_COST && io.terms && T->traj_term >= 0) {
                float tl = 0.f;
                for (int s = 0; s < SLOTS; ++s) tl += sm.tpart[tid * SLOTS + s];
                io.terms[(int64_t)T->traj_term * ld + i] = tl;
            }
            if (io.cost) io.cost[i] = J;
            if (io.mask) io.mask[i] = (uint8_t)m;
            if (MODE == MODE_COST && io.hits) {
                int h = 0;
                for (int s = 0; s < SLOTS; ++s) h += sm.hpart[tid * SLOTS + s];
                io.hits[i] = h;
            }
            if (m) sm.any_sat = 1;
        }
    }
    __syncthreads();
    if (io.first_sat && tid == 0 && sm.any_sat) atomicMin(io.first_sat, iter);

    if (MODE != MODE_COST) {
        // phase 2: sum each coordinate's partials over slots and split lanes
        // in a fixed order, then write G or apply Adam in place
        const float bc1 = 1.f - powf(b1, (float)t), bc2 = 1.f - powf(b2, (float)t);
        const int FQ = 11 + 3 * K;   // foreign-configuration partials
        for (int idx = tid; idx < D * P; idx += WG) {
            const int d = idx / P, p = idx - d * P;
            const int64_t i = p0 + p;
            if (i >= n) continue;
            const int k = d / CT_STEP_DIM, r = d - CT_STEP_DIM * k;
            const float* pp = sm.part + (size_t)p * SLOTS * SPLIT * NP;
            auto lane = [&](int slot, int si) { return pp + (size_t)(slot * SPLIT + si) * NP; };
            float g = 0.f;
#pragma unroll
            for (int si = 0; si < SPLIT; ++si) {
                if (r < 7) {
                    // q_grasp of step k: its slot, plus the start of the holding transition
                    g += lane(2 * k, si)[r] + lane(2 * k + 1, si)[FQ + r];
                } else if (r < 14) {
                    // q_place of step k: its slot, plus the start of the next free transition
                    g += lane(2 * k + 1, si)[r - 7];
                    if (k + 1 < K) g += lane(2 * k + 2, si)[FQ + (r - 7)];
                } else if (r < 18) {
                    g += lane(2 * k, si)[7 + (r - 14)] + lane(2 * k + 1, si)[7 + (r - 14)];
                } else {
                    for (int s = 0; s < SLOTS; ++s) g += lane(s, si)[11 + 3 * k + (r - 18)];
                }
            }
            const int64_t a = d * ld + i;
            if (MODE == MODE_GRAD) {
                io.G[a] = io.gw ? io.gw[i] * g : g;
            } else if (sm.okp[p] && !sm.frz[d]) {
                const float gs = io.gscale * g;
                const float m1 = b1 * sm.ms[idx] + (1.f - b1) * gs;
                const float v1 = b2 * sm.vs[idx] + (1.f - b2) * gs * gs;
                const float mh = m1 / bc1, vh = v1 / bc2;
                io.X[a] = sm.xs[idx] - lr * mh / (sqrtf(vh) + eps);
                io.M[a] = m1;
                io.V[a] = v1;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One skeleton of KT steps: one workgroup per tile (XCD-aware tile order).
template <int SPLIT, int MODE, int KT, bool EXT>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void particle_kernel(
    const Tables* __restrict__ T, float* __restrict__ X, float* __restrict__ M, float* __restrict__ V,
    float* __restrict__ G, float* __restrict__ cost, float* __restrict__ terms, uint8_t* __restrict__ mask,
    int32_t* __restrict__ first_sat, const uint8_t* __restrict__ frozen, int64_t n, int64_t ld, float lr,
    float b1, float b2, float eps, float gscale, int32_t t_arg, const int32_t* __restrict__ t_in,
    int32_t* __restrict__ t_out, int32_t stop_at_first, const float* __restrict__ gw,
    const float* __restrict__ wts, int32_t* __restrict__ hits) {
    __shared__ TileSmem<SPLIT> sm;
    // update number t: explicit, or one past the device counter of applied
    // updates; a captured loop alternates two counter slots (read t_in,
    // write t_out), so no launch writes a slot that its own workgroups read
    const int32_t t = t_in ? *t_in + 1 : t_arg;
    if (t_out && blockIdx.x == 0 && threadIdx.x == 0) *t_out = t;
    // stop-at-first: once an earlier iteration produced a satisfying
    // particle, the remaining steps of a captured loop do nothing (every
    // workgroup reads the same value: this launch only writes iter itself)
    if (stop_at_first && first_sat && *first_sat < t - 1) return;
    // XCD-aware tile order: consecutive workgroups are dealt round-robin to the
    // 8 XCDs, so give each XCD a contiguous range of particle tiles; tiles
    // that share cache lines of X, M and V then share one L2
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const TileIO io{T, X, M, V, G, cost, terms, mask, first_sat, frozen, gw, n, ld, gscale, EXT ? wts : nullptr,
                    stop_at_first ? 1 : 0, MODE == MODE_COST ? hits : nullptr};
    run_tile<KT, SPLIT, MODE, EXT>(io, tile * tile_particles(KT, SPLIT), sm, lr, b1, b2, eps, t);
}


// Many skeletons of different lengths and sizes, one launch per iteration:
// a fixed number of workgroups pull (skeleton, tile) items from a device
// queue (items ordered by cost, largest first) until it is empty; the last
// workgroup to leave resets the queue for the next launch.
template <int SPLIT, bool EXT>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2))) void batch_kernel(const BatchSkel* __restrict__ skels,
                                                   const int2* __restrict__ items, int32_t n_items,
                                                   int32_t* __restrict__ queue, float lr, float b1, float b2,
                                                   float eps, int32_t t_arg, const int32_t* __restrict__ t_in,
                                                   int32_t* __restrict__ t_out) {
    __shared__ TileSmem<SPLIT> sm;
    __shared__ int item_s;
    const int32_t t = t_in ? *t_in + 1 : t_arg;
    if (t_out && blockIdx.x == 0 && threadIdx.x == 0) *t_out = t;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(&queue[0], 1);
        __syncthreads();
        // the item is the same for the whole workgroup: make it wave-uniform
        // so the skeleton's tables are read through the scalar cache
        const int it = __builtin_amdgcn_readfirstlane(item_s);
        __syncthreads();
        if (it >= n_items) break;
        const int2 w = items[it];
        const BatchSkel& b = skels[w.x];
        const TileIO io{b.T, b.X, b.M, b.V, nullptr, b.cost, nullptr, b.mask, b.first_sat, b.frozen, nullptr,
                        b.n, b.ld, b.gscale};
        run_tile<0, SPLIT, MODE_STEP, EXT>(io, (int64_t)w.y * tile_particles(b.T->K, SPLIT), sm, lr, b1, b2, eps, t);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&queue[0], 0);
            atomicExch(&queue[1], 0);
        }
    }
}

}  // namespace ct
