// Host side of the C ABI declared in include/cutamp.h: descriptor validation,
// construction of the device tables of one skeleton's CSP, kernel dispatch,
// the graph-captured optimization loop and the split autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "cutamp.h"
#include "aux_kernels.hpp"
#include "ct_tables.hpp"
#include "pk_dispatch.hpp"

namespace {

struct GraphKey {
    float *X = nullptr, *M = nullptr, *V = nullptr, *cost = nullptr;
    uint8_t* mask = nullptr;
    int32_t* first_sat = nullptr;
    const uint8_t* frozen = nullptr;
    const float* wts = nullptr;
    int64_t n = -1, ld = -1;
    int32_t iters = -1, split = -1, stop = -1;
    float lr = 0, b1 = 0, b2 = 0, eps = 0, gs = 0;
    bool operator==(const GraphKey& o) const {
        return X == o.X && M == o.M && V == o.V && cost == o.cost && mask == o.mask &&
               first_sat == o.first_sat && frozen == o.frozen && wts == o.wts && n == o.n && ld == o.ld &&
               iters == o.iters && split == o.split && stop == o.stop && lr == o.lr && b1 == o.b1 && b2 == o.b2 &&
               eps == o.eps && gs == o.gs;
    }
};

}  // namespace

struct ct_problem {
    ct::Tables h;               // host copy of the tables
    ct::Tables* d = nullptr;    // device copy
    int K = 0, D = 0, n_terms = 0, nc = 0;
    int split = 0;              // 0 = default
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t capture_stream = nullptr;
    hipEvent_t replayed = nullptr;   // recorded after every replay of gexec on the caller's stream
    int32_t* t_dev = nullptr;   // two-slot device counter of applied updates for captured loops,
                                // followed by n_constraint per-constraint counts (feasibility)
    GraphKey key;
    const float* wts = nullptr;  // per-particle term weights (ct_set_term_weights), or null
    int64_t wts_ld = 0;
};

namespace {

bool is_fin(double v) { return std::isfinite(v); }

// A sphere holding every sphere of a set (centre = mean of the centres,
// radius = largest |c_i - centre| + r_i), computed in double from the FP32
// values the kernels use and grown by a relative 1e-6 and 0.1 mm so that an
// FP32 test against it can only err towards "touches".  w = -1: empty set.
float4 bounding_sphere(const float4* sp, int n) {
    if (n <= 0) return make_float4(0.f, 0.f, 0.f, -1.f);
    double c[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        c[0] += sp[i].x;
        c[1] += sp[i].y;
        c[2] += sp[i].z;
    }
    for (double& v : c) v /= n;
    double rad = 0;
    for (int i = 0; i < n; ++i) {
        const double dx = sp[i].x - c[0], dy = sp[i].y - c[1], dz = sp[i].z - c[2];
        rad = std::max(rad, std::sqrt(dx * dx + dy * dy + dz * dz) + (double)sp[i].w);
    }
    return make_float4((float)c[0], (float)c[1], (float)c[2], (float)(rad * (1 + 1e-6) + 1e-4));
}

bool valid_box(const double* b) {
    for (int i = 0; i < 7; ++i)
        if (!is_fin(b[i])) return false;
    return b[4] > 0 && b[5] > 0 && b[6] > 0;
}

ct::SBox to_sbox(const double* b) {
    const double c = std::cos(b[3]), s = std::sin(b[3]);
    ct::SBox o;
    o.c = (float)c;
    o.s = (float)s;
    o.u0 = (float)(-(c * b[0] + s * b[1]));
    o.u1 = (float)(s * b[0] - c * b[1]);
    o.tz = (float)b[2];
    o.hx = (float)b[4];
    o.hy = (float)b[5];
    o.hz = (float)b[6];
    return o;
}

ct::Box to_box(const double* b) {
    ct::Box o;
    o.cx = (float)b[0];
    o.cy = (float)b[1];
    o.cz = (float)b[2];
    o.c = (float)std::cos(b[3]);
    o.s = (float)std::sin(b[3]);
    o.hx = (float)b[4];
    o.hy = (float)b[5];
    o.hz = (float)b[6];
    return o;
}

// Without a tuned choice: the smallest split that gives at least two
// workgroups per compute unit (512 on gfx950's 256 CUs); a workgroup holds
// 256 / (2K split) particles, so the condition is n * 2K * split >= 512 * 256.
int default_split(int K, int64_t n) {
    for (int s = 1; s < 4; s *= 2)
        if (n * 2 * K * s >= int64_t(512) * 256) return s;
    return 4;
}

// n == 0 is an empty batch: only the handle and ld are checked
bool empty_ok(const ct_problem* P, int64_t n, int64_t ld) { return P && n == 0 && ld >= 0 && ld % 64 == 0; }

bool good_layout(const void* p, int64_t n, int64_t ld) {
    if (n < 0 || ld < n || ld % 64 != 0) return false;
    return n == 0 || ((uintptr_t)p % 256) == 0;
}

int err_of(hipError_t e) { return e == hipSuccess ? CT_OK : CT_ERR_DEVICE; }

AdamArgs adam_args(const ct_adam* a) {
    AdamArgs o;
    o.lr = a->lr;
    o.b1 = a->beta1;
    o.b2 = a->beta2;
    o.eps = a->eps;
    o.gs = a->grad_scale;
    return o;
}

bool valid_adam(const ct_adam* a) {
    return a && std::isfinite(a->lr) && a->beta1 >= 0 && a->beta1 < 1 && a->beta2 >= 0 && a->beta2 < 1 &&
           std::isfinite(a->eps) && a->eps >= 0 && std::isfinite(a->grad_scale);
}

// ---------------------------------------------------------------------------
// particle kernel dispatch: split in {1, 2, 4}, with or without the
// self-collision pass (one object file per combination), skeleton length
// K = 1..6, three modes; the many-skeleton kernel reads K from each
// skeleton's tables at run time.  Problems without self-collision run
// kernels that do not contain the pass (it would cost them registers).

PkFn pick_kernel(int split, int K, int mode, bool self) {
    switch (split) {
        case 1: return self ? ct_pick_s1_ext(K, mode) : ct_pick_s1(K, mode);
        case 2: return self ? ct_pick_s2_ext(K, mode) : ct_pick_s2(K, mode);
        case 4: return self ? ct_pick_s4_ext(K, mode) : ct_pick_s4(K, mode);
        default: return nullptr;
    }
}

BatchFn pick_batch(int split, bool self) {
    switch (split) {
        case 1: return self ? ct_batch_s1_ext() : ct_batch_s1();
        case 2: return self ? ct_batch_s2_ext() : ct_batch_s2();
        case 4: return self ? ct_batch_s4_ext() : ct_batch_s4();
        default: return nullptr;
    }
}

int effective_split(const ct_problem* P, int64_t n) { return P->split ? P->split : default_split(P->K, n); }

// One launch of the particle kernel for problem P.  `weighted`: apply the
// problem's per-particle term weights if it has any (their ld must be the
// call's); the many-skeleton reference launches pass false.
int run_pk(const ct_problem* P, int mode, const PkArgs& a, hipStream_t st, int split = 0, bool weighted = true) {
    if (a.n == 0) return CT_OK;
    PkArgs b = a;
    b.wts = weighted ? P->wts : nullptr;
    if (b.wts && P->wts_ld != a.ld) return CT_ERR_INVALID_ARG;
    PkFn f = pick_kernel(split ? split : effective_split(P, a.n), P->K, mode, P->h.self_on || b.wts);
    if (!f) return CT_ERR_UNSUPPORTED;
    return err_of(f(P->d, b, st));
}

// A graph exec must not be destroyed while a replay of it is still queued or
// running: its kernel-argument storage is released with it, and the queued
// dispatches (and a profiler's completion handler reading them) would then
// touch freed memory.  Every replay records `replayed` on the caller's
// stream; dropping the graph first waits for that event.
void drop_graph(ct_problem* P) {
    if (P->gexec && P->replayed) hipEventSynchronize(P->replayed);
    if (P->gexec) hipGraphExecDestroy(P->gexec);
    if (P->graph) hipGraphDestroy(P->graph);
    P->gexec = nullptr;
    P->graph = nullptr;
    P->key = GraphKey();
}

}  // namespace

// ===========================================================================

extern "C" const char* ct_status_string(int status) {
    switch (status) {
        case CT_OK: return "ok";
        case CT_ERR_INVALID_ARG: return "invalid argument";
        case CT_ERR_UNSUPPORTED: return "unsupported by this library";
        case CT_ERR_ALLOC: return "device allocation failed";
        case CT_ERR_DEVICE: return "HIP runtime or kernel launch failure";
        default: return "unknown status";
    }
}

extern "C" int ct_problem_create(const ct_robot* robot, const ct_scene* scene, const ct_skeleton* sk,
                                 const ct_weights* w, const ct_tolerances* e, ct_problem** out) {
    if (!out) return CT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!robot || !scene || !sk || !w || !e) return CT_ERR_INVALID_ARG;
    // ---- robot
    if (robot->n_joints != CT_N_JOINTS) return CT_ERR_UNSUPPORTED;
    if (!robot->dh || !robot->q_lo || !robot->q_hi || !robot->spheres || !robot->sphere_link)
        return CT_ERR_INVALID_ARG;
    if (robot->n_spheres < 1) return CT_ERR_INVALID_ARG;
    if (robot->n_spheres > CT_MAX_ROBOT_SPHERES) return CT_ERR_UNSUPPORTED;
    for (int i = 0; i < 4 * CT_N_JOINTS; ++i)
        if (!is_fin(robot->dh[i])) return CT_ERR_INVALID_ARG;
    for (int i = 0; i < CT_N_JOINTS; ++i)
        if (!is_fin(robot->q_lo[i]) || !is_fin(robot->q_hi[i]) || !(robot->q_lo[i] < robot->q_hi[i]))
            return CT_ERR_INVALID_ARG;
    if (!is_fin(robot->tool_d)) return CT_ERR_INVALID_ARG;
    for (int s = 0; s < robot->n_spheres; ++s) {
        for (int c = 0; c < 4; ++c)
            if (!is_fin(robot->spheres[4 * s + c])) return CT_ERR_INVALID_ARG;
        if (!(robot->spheres[4 * s + 3] > 0)) return CT_ERR_INVALID_ARG;
        if (robot->sphere_link[s] < 1 || robot->sphere_link[s] > 8) return CT_ERR_INVALID_ARG;
    }
    // ---- scene
    if (!scene->table || !valid_box(scene->table)) return CT_ERR_INVALID_ARG;
    if (scene->n_obstacles < 0 || (scene->n_obstacles > 0 && !scene->obstacles)) return CT_ERR_INVALID_ARG;
    for (int b = 0; b < scene->n_obstacles; ++b)
        if (!valid_box(scene->obstacles + 7 * b)) return CT_ERR_INVALID_ARG;
    if (scene->n_objects < 1 || !scene->objects || !scene->obj_spheres) return CT_ERR_INVALID_ARG;
    if (scene->n_objects > CT_MAX_OBJECTS) return CT_ERR_UNSUPPORTED;
    for (int o = 0; o < scene->n_objects; ++o)
        if (!valid_box(scene->objects + 7 * o)) return CT_ERR_INVALID_ARG;
    if (scene->n_obj_spheres < 1) return CT_ERR_INVALID_ARG;
    if (scene->n_obj_spheres > CT_MAX_OBJ_SPHERES) return CT_ERR_UNSUPPORTED;
    for (int i = 0; i < scene->n_objects * scene->n_obj_spheres; ++i) {
        for (int c = 0; c < 4; ++c)
            if (!is_fin(scene->obj_spheres[4 * i + c])) return CT_ERR_INVALID_ARG;
        if (!(scene->obj_spheres[4 * i + 3] > 0)) return CT_ERR_INVALID_ARG;
    }
    for (int c = 0; c < 2; ++c)
        if (!is_fin(scene->region_lo[c]) || !is_fin(scene->region_hi[c]) ||
            !(scene->region_lo[c] < scene->region_hi[c]))
            return CT_ERR_INVALID_ARG;
    // ---- skeleton
    const int K = sk->n_steps;
    if (K < 1) return CT_ERR_INVALID_ARG;
    if (K > CT_MAX_STEPS) return CT_ERR_UNSUPPORTED;
    if (!sk->object_of_step || !sk->grasp_lo || !sk->grasp_hi) return CT_ERR_INVALID_ARG;
    if (sk->goal_cost != 0 && sk->goal_cost != 1) return CT_ERR_INVALID_ARG;
    if (sk->self_collision != 0 && sk->self_collision != 1) return CT_ERR_INVALID_ARG;
    if (sk->waypoints < 0) return CT_ERR_INVALID_ARG;
    if (sk->waypoints > CT_MAX_WAYPOINTS) return CT_ERR_UNSUPPORTED;
    if (sk->waypoints > 0) {
        if (!sk->q0) return CT_ERR_INVALID_ARG;
        for (int j = 0; j < CT_N_JOINTS; ++j)
            if (!is_fin(sk->q0[j])) return CT_ERR_INVALID_ARG;
    }
    std::vector<int> used(scene->n_objects, 0);
    for (int k = 0; k < K; ++k) {
        const int o = sk->object_of_step[k];
        if (o < 0 || o >= scene->n_objects || used[o]) return CT_ERR_INVALID_ARG;
        used[o] = 1;
        for (int c = 0; c < 3; ++c)
            if (!is_fin(sk->grasp_lo[3 * k + c]) || !is_fin(sk->grasp_hi[3 * k + c]) ||
                sk->grasp_lo[3 * k + c] > sk->grasp_hi[3 * k + c])
                return CT_ERR_INVALID_ARG;
    }
    const int n_unmoved = scene->n_objects - K;
    if (1 + scene->n_obstacles + n_unmoved > CT_MAX_STATIC_BOXES) return CT_ERR_UNSUPPORTED;
    // ---- weights and tolerances
    const double ws[ct::W_N] = {w->kin_pos, w->kin_rot, w->grasp,       w->place,       w->jlim,
                                w->coll,    w->goal,    w->traj_len,    w->motion_coll, w->self_coll};
    for (double v : ws)
        if (!is_fin(v) || v < 0) return CT_ERR_INVALID_ARG;
    const double es[ct::E_N] = {e->kin_pos, e->kin_rot, e->grasp,       e->place,
                                e->jlim,    e->coll,    e->motion_coll, e->self_coll};
    for (double v : es)
        if (!is_fin(v) || v < 0) return CT_ERR_INVALID_ARG;

    ct_problem* P = new (std::nothrow) ct_problem();
    if (!P) return CT_ERR_ALLOC;
    ct::Tables& T = P->h;
    std::memset(&T, 0, sizeof(T));
    T.K = K;
    T.D = CT_STEP_DIM * K;
    T.W = sk->waypoints;
    T.self_on = sk->self_collision;
    T.self_term = T.self_on ? CT_TERMS_PER_STEP * K + (T.W > 0 ? 2 * K : 0) : -1;
    T.n_constraint = CT_TERMS_PER_STEP * K + (T.W > 0 ? 2 * K : 0) + (T.self_on ? 2 * K : 0);
    T.goal = sk->goal_cost;
    T.goal_term = T.goal ? T.n_constraint : -1;
    T.traj_term = T.W > 0 ? T.n_constraint + T.goal : -1;
    T.n_terms = T.n_constraint + T.goal + (T.W > 0 ? 1 : 0);
    T.n_os = scene->n_obj_spheres;
    for (int i = 0; i < CT_N_JOINTS; ++i) {
        const double* r = robot->dh + 4 * i;
        T.a[i] = (float)r[0];
        T.ca[i] = (float)std::cos(r[1]);
        T.sa[i] = (float)std::sin(r[1]);
        T.d[i] = (float)r[2];
        T.th0[i] = (float)r[3];
        T.q_lo[i] = (float)robot->q_lo[i];
        T.q_hi[i] = (float)robot->q_hi[i];
        T.q0[i] = sk->q0 ? (float)sk->q0[i] : 0.f;
    }
    T.tool_d = (float)robot->tool_d;
    // robot spheres grouped by link (stable within a link)
    int cnt = 0;
    T.link_start[0] = T.link_start[1] = 0;
    for (int L = 1; L <= 8; ++L) {
        T.link_start[L] = cnt;
        for (int s = 0; s < robot->n_spheres; ++s)
            if (robot->sphere_link[s] == L) {
                const double* sp = robot->spheres + 4 * s;
                T.rs[cnt++] = make_float4((float)sp[0], (float)sp[1], (float)sp[2], (float)sp[3]);
            }
    }
    T.link_start[9] = cnt;
    for (int L = 0; L < 10; ++L)
        T.lbs[L] = (L >= 1 && L <= 8) ? bounding_sphere(T.rs + T.link_start[L], T.link_start[L + 1] - T.link_start[L])
                                      : make_float4(0.f, 0.f, 0.f, -1.f);
    // boxes that never move
    int nb = 0;
    T.sbox[nb++] = to_sbox(scene->table);
    for (int b = 0; b < scene->n_obstacles; ++b) T.sbox[nb++] = to_sbox(scene->obstacles + 7 * b);
    for (int o = 0; o < scene->n_objects; ++o)
        if (!used[o]) T.sbox[nb++] = to_sbox(scene->objects + 7 * o);
    T.n_static = nb;
    const double table_top = scene->table[2] + scene->table[6];
    for (int k = 0; k < K; ++k) {
        const int o = sk->object_of_step[k];
        const double* ob = scene->objects + 7 * o;
        T.obj0[k] = to_box(ob);
        T.p0_yaw[k] = (float)ob[3];
        T.place_z[k] = (float)(table_top + ob[6]);
        for (int c = 0; c < 3; ++c) {
            T.grasp_lo[k][c] = (float)sk->grasp_lo[3 * k + c];
            T.grasp_hi[k][c] = (float)sk->grasp_hi[3 * k + c];
        }
        for (int m = 0; m < T.n_os; ++m) {
            const double* sp = scene->obj_spheres + 4 * (o * T.n_os + m);
            T.os[k][m] = make_float4((float)sp[0], (float)sp[1], (float)sp[2], (float)sp[3]);
        }
        T.obs[k] = bounding_sphere(T.os[k], T.n_os);
        // uniform-initialization box of step k's 21 coordinates
        float* lo = T.lo + CT_STEP_DIM * k;
        float* hi = T.hi + CT_STEP_DIM * k;
        for (int j = 0; j < 7; ++j) {
            lo[j] = lo[7 + j] = (float)robot->q_lo[j];
            hi[j] = hi[7 + j] = (float)robot->q_hi[j];
        }
        for (int c = 0; c < 3; ++c) {
            lo[14 + c] = (float)sk->grasp_lo[3 * k + c];
            hi[14 + c] = (float)sk->grasp_hi[3 * k + c];
        }
        lo[17] = lo[20] = (float)-M_PI;
        hi[17] = hi[20] = (float)M_PI;
        lo[18] = (float)scene->region_lo[0];
        hi[18] = (float)scene->region_hi[0];
        lo[19] = (float)scene->region_lo[1];
        hi[19] = (float)scene->region_hi[1];
    }
    for (int c = 0; c < 2; ++c) {
        T.region_lo[c] = (float)scene->region_lo[c];
        T.region_hi[c] = (float)scene->region_hi[c];
    }
    for (int i = 0; i < ct::W_N; ++i) T.w[i] = (float)ws[i];
    for (int i = 0; i < ct::E_N; ++i) T.eps[i] = (float)es[i];

    P->K = K;
    P->D = T.D;
    P->n_terms = T.n_terms;
    P->nc = T.n_constraint;
    if (hipMalloc(&P->d, sizeof(ct::Tables)) != hipSuccess) {
        delete P;
        return CT_ERR_ALLOC;
    }
    if (hipMalloc(&P->t_dev, (2 + (size_t)P->nc) * sizeof(int32_t)) != hipSuccess) {
        hipFree(P->d);
        delete P;
        return CT_ERR_ALLOC;
    }
    if (hipMemcpy(P->d, &T, sizeof(ct::Tables), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(P->d);
        hipFree(P->t_dev);
        delete P;
        return CT_ERR_DEVICE;
    }
    *out = P;
    return CT_OK;
}

extern "C" int ct_problem_destroy(ct_problem* P) {
    if (!P) return CT_OK;
    // eager launches on any stream may still read the tables and counters
    hipDeviceSynchronize();
    drop_graph(P);
    if (P->replayed) hipEventDestroy(P->replayed);
    if (P->capture_stream) hipStreamDestroy(P->capture_stream);
    if (P->d) hipFree(P->d);
    if (P->t_dev) hipFree(P->t_dev);
    delete P;
    return CT_OK;
}

extern "C" int ct_set_term_weights(ct_problem* P, const float* W, int64_t ld) {
    if (!P) return CT_ERR_INVALID_ARG;
    if (W && (ld <= 0 || !good_layout(W, 1, ld))) return CT_ERR_INVALID_ARG;
    if (W != P->wts || (W && ld != P->wts_ld)) drop_graph(P);   // a captured loop holds the old pointer
    P->wts = W;
    P->wts_ld = W ? ld : 0;
    return CT_OK;
}

extern "C" int ct_al_update(const ct_problem* P, const float* terms, int64_t n, int64_t ld, float rho, float* mu,
                            float* W, void* stream) {
    if (empty_ok(P, n, ld) && std::isfinite(rho) && rho >= 0) return CT_OK;
    if (!P || !terms || !mu || !W || !std::isfinite(rho) || rho < 0) return CT_ERR_INVALID_ARG;
    if (!good_layout(terms, n, ld) || !good_layout(mu, n, ld) || !good_layout(W, n, ld)) return CT_ERR_INVALID_ARG;
    if (n == 0) return CT_OK;
    const int64_t total = (int64_t)P->n_terms * n;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(ct::al_update_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, P->d, terms, n, ld,
                       rho, mu, W);
    return err_of(hipGetLastError());
}

extern "C" int ct_al_weights(const ct_problem* P, const float* terms, int64_t n, int64_t ld, float rho,
                             const float* mu, float* W, void* stream) {
    if (empty_ok(P, n, ld) && std::isfinite(rho) && rho >= 0) return CT_OK;
    if (!P || !terms || !mu || !W || !std::isfinite(rho) || rho < 0) return CT_ERR_INVALID_ARG;
    if (!good_layout(terms, n, ld) || !good_layout(mu, n, ld) || !good_layout(W, n, ld)) return CT_ERR_INVALID_ARG;
    if (n == 0) return CT_OK;
    const int64_t total = (int64_t)P->n_terms * n;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(ct::al_weights_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, P->d, terms, n, ld,
                       rho, mu, W);
    return err_of(hipGetLastError());
}

extern "C" int ct_feasibility(const ct_problem* P, const float* terms, int64_t n, int64_t ld, float penalty,
                              int32_t* counts, float* H, void* stream) {
    if (!P || !std::isfinite(penalty)) return CT_ERR_INVALID_ARG;
    if (n < 0 || ld < n || ld % 64 != 0 || (n > 0 && !terms)) return CT_ERR_INVALID_ARG;
    if (terms && ((uintptr_t)terms % 256)) return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    int32_t* cnt = counts ? counts : P->t_dev + 2;
    hipLaunchKernelGGL(ct::feas_count_kernel, dim3(P->nc), dim3(256), 0, st, P->d, terms, n, ld, cnt);
    if (H) hipLaunchKernelGGL(ct::feas_h_kernel, dim3(1), dim3(64), 0, st, cnt, P->nc, penalty, H);
    return err_of(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Allocation-free feasibility: the per-constraint counts live in one
// file-scope device array per GPU (held until the process ends) instead of
// the handle's buffer.  Host code never passes `scratch` itself to a kernel
// (in host code the name is a stand-in, not a device address): the address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and is kept per device.

static __device__ __align__(256) int32_t scratch[CT_FEAS_SCRATCH_MAX];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};

int device_scratch(int32_t** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CT_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CT_ERR_DEVICE;
        g_scratch_ptr[dev] = (int32_t*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return CT_OK;
}

}  // namespace

extern "C" int ct_feasibility_noalloc(const ct_problem* P, const float* terms, int64_t n, int64_t ld, float penalty,
                                      float* H, void* stream) {
    if (!P || !H || !std::isfinite(penalty)) return CT_ERR_INVALID_ARG;
    if (n < 0 || ld < n || ld % 64 != 0 || (n > 0 && !terms)) return CT_ERR_INVALID_ARG;
    if (terms && ((uintptr_t)terms % 256)) return CT_ERR_INVALID_ARG;
    if (P->nc > CT_FEAS_SCRATCH_MAX) return CT_ERR_UNSUPPORTED;
    int32_t* cnt = nullptr;
    const int rc = device_scratch(&cnt);
    if (rc != CT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    // every count is written (not accumulated), so nothing needs clearing
    hipLaunchKernelGGL(ct::feas_count_kernel, dim3(P->nc), dim3(256), 0, st, P->d, terms, n, ld, cnt);
    hipLaunchKernelGGL(ct::feas_h_kernel, dim3(1), dim3(64), 0, st, cnt, P->nc, penalty, H);
    return err_of(hipGetLastError());
}

extern "C" int ct_step_mask(const ct_problem* P, const float* terms, int64_t n, int64_t ld, uint8_t* step_mask,
                            int64_t ld_mask, int32_t* count, void* stream) {
    if (!P || n < 0 || ld < n || ld % 64 != 0 || (n > 0 && !terms)) return CT_ERR_INVALID_ARG;
    if (terms && ((uintptr_t)terms % 256)) return CT_ERR_INVALID_ARG;
    if (step_mask && ld_mask < n) return CT_ERR_INVALID_ARG;
    if (n == 0 || (!step_mask && !count)) return CT_OK;
    hipLaunchKernelGGL(ct::step_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       P->d, terms, n, ld, step_mask, ld_mask, count);
    return err_of(hipGetLastError());
}

extern "C" int ct_compact(const uint8_t* mask, int64_t n, int32_t* idx, int32_t* count, void* stream) {
    if (n < 0 || n > INT32_MAX || !count || (n > 0 && (!mask || !idx))) return CT_ERR_INVALID_ARG;
    hipLaunchKernelGGL(ct::compact_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, mask, n, idx, count);
    return err_of(hipGetLastError());
}

extern "C" int ct_gather_block(const float* Xs, int64_t lds, int32_t rows, int64_t n_src, const int32_t* idx,
                               const int32_t* count, float* X, float* M, float* V, int64_t ld, int32_t row0,
                               int64_t n, void* stream) {
    if (rows < 0 || row0 < 0 || n < 0 || ld < n || ld % 64 != 0 || n_src < 0 || lds < n_src) return CT_ERR_INVALID_ARG;
    if (n == 0 || rows == 0) return CT_OK;
    if (!Xs || !X || n_src == 0 || (count && !idx)) return CT_ERR_INVALID_ARG;
    hipLaunchKernelGGL(ct::gather_block_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       Xs, lds, rows, idx, count, n_src, X, M, V, ld, row0, n);
    return err_of(hipGetLastError());
}

extern "C" int ct_problem_info(const ct_problem* P, int32_t* dim, int32_t* n_terms, int32_t* n_constraint) {
    if (!P) return CT_ERR_INVALID_ARG;
    if (dim) *dim = P->D;
    if (n_terms) *n_terms = P->n_terms;
    if (n_constraint) *n_constraint = P->nc;
    return CT_OK;
}

extern "C" int ct_seed_uniform(const ct_problem* P, uint64_t seed, float* X, float* M, float* V, int64_t n,
                               int64_t ld, void* stream) {
    if (empty_ok(P, n, ld)) return CT_OK;
    if (!P || !X || !good_layout(X, n, ld)) return CT_ERR_INVALID_ARG;
    if ((M && !good_layout(M, n, ld)) || (V && !good_layout(V, n, ld))) return CT_ERR_INVALID_ARG;
    if (n == 0) return CT_OK;
    const dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(ct::seed_uniform_kernel, grid, dim3(256), 0, (hipStream_t)stream, P->d,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), X, M, V, n, ld);
    return err_of(hipGetLastError());
}

extern "C" int ct_seed_sampled(const ct_problem* P, uint64_t seed, float* X, float* M, float* V, int64_t n,
                               int64_t ld, void* stream) {
    const int rc = ct_seed_uniform(P, seed, X, M, V, n, ld, stream);
    if (rc != CT_OK || n == 0) return rc;
    hipLaunchKernelGGL(ct::place_sampler_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       P->d, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), X, n, ld);
    return err_of(hipGetLastError());
}

extern "C" int ct_cost(const ct_problem* P, const float* X, int64_t n, int64_t ld, float* cost, float* terms,
                       uint8_t* mask, void* stream) {
    if (empty_ok(P, n, ld)) return CT_OK;
    if (!P || !X || !cost || !good_layout(X, n, ld)) return CT_ERR_INVALID_ARG;
    if (terms && !good_layout(terms, n, ld)) return CT_ERR_INVALID_ARG;
    PkArgs a{};
    a.X = const_cast<float*>(X);
    a.cost = cost;
    a.terms = terms;
    a.mask = mask;
    a.n = n;
    a.ld = ld;
    return run_pk(P, ct::MODE_COST, a, (hipStream_t)stream);
}

extern "C" int ct_penetrating_pairs(const ct_problem* P, const float* X, int64_t n, int64_t ld, int32_t* pairs,
                                    void* stream) {
    if (empty_ok(P, n, ld)) return CT_OK;
    if (!P || !X || !pairs || !good_layout(X, n, ld)) return CT_ERR_INVALID_ARG;
    PkArgs a{};
    a.X = const_cast<float*>(X);
    a.n = n;
    a.ld = ld;
    a.hits = pairs;
    return run_pk(P, ct::MODE_COST, a, (hipStream_t)stream);
}

extern "C" int ct_cost_grad(const ct_problem* P, const float* X, int64_t n, int64_t ld, float* cost, float* G,
                            const float* weights, void* stream) {
    if (empty_ok(P, n, ld)) return CT_OK;
    if (!P || !X || !G || !good_layout(X, n, ld) || !good_layout(G, n, ld)) return CT_ERR_INVALID_ARG;
    PkArgs a{};
    a.X = const_cast<float*>(X);
    a.G = G;
    a.cost = cost;
    a.gw = weights;
    a.n = n;
    a.ld = ld;
    return run_pk(P, ct::MODE_GRAD, a, (hipStream_t)stream);
}

extern "C" int ct_adam_apply(const ct_problem* P, float* X, float* M, float* V, const float* G, int64_t n,
                             int64_t ld, int64_t t, const ct_adam* adam, const uint8_t* frozen, void* stream) {
    if (empty_ok(P, n, ld)) return CT_OK;
    if (!P || !X || !M || !V || !G || t < 1 || !valid_adam(adam)) return CT_ERR_INVALID_ARG;
    if (!good_layout(X, n, ld) || !good_layout(M, n, ld) || !good_layout(V, n, ld) || !good_layout(G, n, ld))
        return CT_ERR_INVALID_ARG;
    if (n == 0) return CT_OK;
    const AdamArgs a = adam_args(adam);
    const dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(ct::adam_kernel, grid, dim3(256), 0, (hipStream_t)stream, P->D, X, M, V, G, frozen, n, ld,
                       a.lr, a.b1, a.b2, a.eps, a.gs, (int32_t)t);
    return err_of(hipGetLastError());
}

namespace {
int step_impl(const ct_problem* P, float* X, float* M, float* V, int64_t n, int64_t ld, int64_t t,
              const ct_adam* adam, const uint8_t* frozen, float* cost, uint8_t* mask, int32_t* first_sat,
              hipStream_t st, int split, const int32_t* t_in = nullptr, int32_t* t_out = nullptr,
              int32_t stop_at_first = 0) {
    PkArgs a{};
    a.X = X;
    a.M = M;
    a.V = V;
    a.cost = cost;
    a.mask = mask;
    a.first_sat = first_sat;
    a.frozen = frozen;
    a.n = n;
    a.ld = ld;
    a.a = adam_args(adam);
    a.t = (int32_t)t;
    a.t_in = t_in;
    a.t_out = t_out;
    a.stop_at_first = stop_at_first;
    return run_pk(P, ct::MODE_STEP, a, st, split);
}

bool valid_step_args(const ct_problem* P, float* X, float* M, float* V, int64_t n, int64_t ld,
                     const ct_adam* adam) {
    return P && X && M && V && valid_adam(adam) && good_layout(X, n, ld) && good_layout(M, n, ld) &&
           good_layout(V, n, ld);
}
}  // namespace

extern "C" int ct_step(const ct_problem* P, float* X, float* M, float* V, int64_t n, int64_t ld, int64_t t,
                       const ct_adam* adam, const uint8_t* frozen, float* cost, uint8_t* mask,
                       int32_t* first_sat, void* stream) {
    if (empty_ok(P, n, ld) && t >= 1) return CT_OK;
    if (!valid_step_args(P, X, M, V, n, ld, adam) || t < 1) return CT_ERR_INVALID_ARG;
    return step_impl(P, X, M, V, n, ld, t, adam, frozen, cost, mask, first_sat, (hipStream_t)stream, 0);
}

extern "C" int ct_optimize(ct_problem* P, float* X, float* M, float* V, int64_t n, int64_t ld, int64_t t0,
                           int32_t iters, const ct_adam* adam, const uint8_t* frozen, float* cost, uint8_t* mask,
                           int32_t* first_sat, int32_t stop_at_first, void* stream) {
    if (empty_ok(P, n, ld) && t0 >= 0 && iters >= 0) return CT_OK;
    if (!valid_step_args(P, X, M, V, n, ld, adam) || t0 < 0 || iters < 0 || t0 + iters > INT32_MAX)
        return CT_ERR_INVALID_ARG;
    if (stop_at_first && !first_sat) return CT_ERR_INVALID_ARG;
    if (n == 0 || iters == 0) return CT_OK;
    GraphKey key;
    key.X = X; key.M = M; key.V = V; key.cost = cost; key.mask = mask; key.first_sat = first_sat;
    key.frozen = frozen; key.wts = P->wts; key.n = n; key.ld = ld; key.iters = iters;
    key.split = effective_split(P, n);
    key.stop = stop_at_first ? 1 : 0;
    key.lr = adam->lr; key.b1 = adam->beta1; key.b2 = adam->beta2; key.eps = adam->eps;
    key.gs = adam->grad_scale;
    if (!(P->gexec && P->key == key)) {
        // capture iters steps; the update number comes from the device
        // counter (two slots used alternately), so one graph serves every t0
        drop_graph(P);
        if (!P->capture_stream && hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return CT_ERR_DEVICE;
        if (hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return CT_ERR_DEVICE;
        int rc = CT_OK;
        for (int32_t it = 0; it < iters && rc == CT_OK; ++it) {
            rc = step_impl(P, X, M, V, n, ld, 0, adam, frozen, cost, mask, first_sat, P->capture_stream, key.split,
                           P->t_dev + (it & 1), P->t_dev + ((it + 1) & 1), key.stop);
        }
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(P->capture_stream, &g);
        if (rc != CT_OK || ec != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            return rc != CT_OK ? rc : CT_ERR_DEVICE;
        }
        hipGraphExec_t ge = nullptr;
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            return CT_ERR_DEVICE;
        }
        P->graph = g;
        P->gexec = ge;
        P->key = key;
    }
    if (!P->replayed && hipEventCreateWithFlags(&P->replayed, hipEventDisableTiming) != hipSuccess) {
        P->replayed = nullptr;
        return CT_ERR_DEVICE;
    }
    hipLaunchKernelGGL(ct::counter_set_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream, P->t_dev, (int32_t)t0);
    int rc = err_of(hipGetLastError());
    if (rc != CT_OK) return rc;
    rc = err_of(hipGraphLaunch(P->gexec, (hipStream_t)stream));
    if (rc != CT_OK) return rc;
    return err_of(hipEventRecord(P->replayed, (hipStream_t)stream));
}

extern "C" int ct_set_split(ct_problem* P, int32_t split) {
    if (!P || !(split == 0 || split == 1 || split == 2 || split == 4)) return CT_ERR_INVALID_ARG;
    if (split != P->split) drop_graph(P);
    P->split = split;
    return CT_OK;
}

extern "C" int ct_get_split(const ct_problem* P, int32_t* split) {
    if (!P || !split) return CT_ERR_INVALID_ARG;
    *split = P->split;
    return CT_OK;
}

extern "C" int ct_autotune(ct_problem* P, const float* X, int64_t n, int64_t ld, int32_t* chosen, void* stream) {
    if (!P || !X || !good_layout(X, n, ld) || n == 0) return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = (size_t)P->D * (size_t)ld * sizeof(float);
    float *Xs = nullptr, *Ms = nullptr, *Vs = nullptr;
    if (hipMalloc(&Xs, bytes) != hipSuccess || hipMalloc(&Ms, bytes) != hipSuccess ||
        hipMalloc(&Vs, bytes) != hipSuccess) {
        hipFree(Xs);
        hipFree(Ms);
        hipFree(Vs);
        return CT_ERR_ALLOC;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    const ct_adam adam{1e-2f, 0.9f, 0.999f, 1e-8f, 1.f / (float)n};
    const int cands[3] = {1, 2, 4};
    float best = 1e30f;
    int best_split = default_split(P->K, n);
    int rc = CT_OK;
    for (int c : cands) {
        if (hipMemcpyAsync(Xs, X, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) { rc = CT_ERR_DEVICE; break; }
        hipMemsetAsync(Ms, 0, bytes, st);
        hipMemsetAsync(Vs, 0, bytes, st);
        for (int w = 0; w < 2 && rc == CT_OK; ++w)
            rc = step_impl(P, Xs, Ms, Vs, n, ld, 1 + w, &adam, nullptr, nullptr, nullptr, nullptr, st, c);
        hipEventRecord(e0, st);
        const int reps = 10;
        for (int r = 0; r < reps && rc == CT_OK; ++r)
            rc = step_impl(P, Xs, Ms, Vs, n, ld, 3 + r, &adam, nullptr, nullptr, nullptr, nullptr, st, c);
        hipEventRecord(e1, st);
        if (rc != CT_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) { rc = CT_ERR_DEVICE; break; }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            best_split = c;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamSynchronize(st);
    hipFree(Xs);
    hipFree(Ms);
    hipFree(Vs);
    if (rc != CT_OK) return rc;
    ct_set_split(P, best_split);
    if (chosen) *chosen = best_split;
    return CT_OK;
}

// ===========================================================================
// many skeletons

struct ct_batch {
    std::vector<ct_problem*> probs;
    std::vector<ct::BatchSkel> skels;   // host copy
    ct::BatchSkel* d_skels = nullptr;
    int2* d_items = nullptr;
    int32_t n_items = 0;
    int32_t* d_queue = nullptr;   // [0] next item, [1] workgroups done
    int32_t* t_dev = nullptr;     // two-slot step counter
    int split = 0, workgroups = 0, persistent = 1;
    int n_cu = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t capture_stream = nullptr;
    hipEvent_t replayed = nullptr;   // recorded after every replay of gexec (see drop_graph)
    int32_t g_iters = -1, g_split = -1, g_wg = -1, g_pers = -1;
    float g_lr = 0, g_b1 = 0, g_b2 = 0, g_eps = 0;
};

namespace {

void batch_drop_graph(ct_batch* B) {
    if (B->gexec && B->replayed) hipEventSynchronize(B->replayed);
    if (B->gexec) hipGraphExecDestroy(B->gexec);
    if (B->graph) hipGraphDestroy(B->graph);
    B->gexec = nullptr;
    B->graph = nullptr;
    B->g_iters = -1;
}

int batch_split(const ct_batch* B) { return B->split ? B->split : 1; }
int batch_workgroups(const ct_batch* B) { return B->workgroups ? B->workgroups : 2 * B->n_cu; }

// (skeleton, tile) items for the current split, largest tiles first: a tile's
// work grows with the boxes each of its configurations is tested against
int batch_build_items(ct_batch* B) {
    const int split = batch_split(B);
    std::vector<std::pair<int, int2>> items;
    for (size_t s = 0; s < B->probs.size(); ++s) {
        const ct_problem* P = B->probs[s];
        const int per = ct::tile_particles(P->K, split);
        const int64_t tiles = (B->skels[s].n + per - 1) / per;
        const int w = P->h.n_static + P->K - 1 + 2 * P->h.W * 1;
        for (int64_t t = 0; t < tiles; ++t) items.push_back({w, make_int2((int)s, (int)t)});
    }
    std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    std::vector<int2> flat(items.size());
    for (size_t i = 0; i < items.size(); ++i) flat[i] = items[i].second;
    if (B->d_items) hipFree(B->d_items);
    B->d_items = nullptr;
    B->n_items = (int32_t)flat.size();
    if (flat.empty()) return CT_OK;
    if (hipMalloc(&B->d_items, flat.size() * sizeof(int2)) != hipSuccess) return CT_ERR_ALLOC;
    if (hipMemcpy(B->d_items, flat.data(), flat.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        return CT_ERR_DEVICE;
    return CT_OK;
}

int batch_launch(ct_batch* B, const ct_adam* adam, int32_t t, const int32_t* t_in, int32_t* t_out, hipStream_t st) {
    AdamArgs a = adam_args(adam);
    if (B->persistent) {
        if (B->n_items == 0) return CT_OK;
        bool self = false;
        for (const ct_problem* P : B->probs) self = self || P->h.self_on;
        BatchFn f = pick_batch(batch_split(B), self);
        if (!f) return CT_ERR_UNSUPPORTED;
        BatchArgs g{};
        g.skels = B->d_skels;
        g.items = B->d_items;
        g.n_items = B->n_items;
        g.queue = B->d_queue;
        g.n_workgroups = batch_workgroups(B);
        g.a = a;
        g.t = t;
        g.t_in = t_in;
        g.t_out = t_out;
        return err_of(f(g, st));
    }
    // reference point: one ordinary launch per skeleton; every launch reads
    // the same counter slot and only the last writes the next one
    for (size_t s = 0; s < B->probs.size(); ++s) {
        const ct::BatchSkel& k = B->skels[s];
        if (k.n == 0) continue;
        PkArgs p{};
        p.X = k.X; p.M = k.M; p.V = k.V; p.cost = k.cost; p.mask = k.mask; p.first_sat = k.first_sat;
        p.frozen = k.frozen; p.n = k.n; p.ld = k.ld; p.a = a; p.a.gs = k.gscale; p.t = t; p.t_in = t_in;
        p.t_out = (s + 1 == B->probs.size()) ? t_out : nullptr;
        const int rc = run_pk(B->probs[s], ct::MODE_STEP, p, st, batch_split(B), false);
        if (rc != CT_OK) return rc;
    }
    return CT_OK;
}

}  // namespace

extern "C" int ct_batch_create(int32_t count, ct_problem* const* problems, float* const* X, float* const* M,
                               float* const* V, const int64_t* n, const int64_t* ld, float* const* cost,
                               uint8_t* const* mask, int32_t* const* first_sat, const uint8_t* const* frozen,
                               ct_batch** out) {
    if (!out) return CT_ERR_INVALID_ARG;
    *out = nullptr;
    if (count < 1 || !problems || !X || !M || !V || !n || !ld) return CT_ERR_INVALID_ARG;
    for (int s = 0; s < count; ++s) {
        if (!problems[s] || !X[s] || !M[s] || !V[s]) return CT_ERR_INVALID_ARG;
        if (!good_layout(X[s], n[s], ld[s]) || !good_layout(M[s], n[s], ld[s]) || !good_layout(V[s], n[s], ld[s]))
            return CT_ERR_INVALID_ARG;
        if (n[s] > INT32_MAX) return CT_ERR_UNSUPPORTED;
    }
    ct_batch* B = new (std::nothrow) ct_batch();
    if (!B) return CT_ERR_ALLOC;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        B->n_cu = prop.multiProcessorCount;
    for (int s = 0; s < count; ++s) {
        ct::BatchSkel k{};
        k.T = problems[s]->d;
        k.X = X[s]; k.M = M[s]; k.V = V[s];
        k.cost = cost ? cost[s] : nullptr;
        k.mask = mask ? mask[s] : nullptr;
        k.first_sat = first_sat ? first_sat[s] : nullptr;
        k.frozen = frozen ? frozen[s] : nullptr;
        k.n = n[s];
        k.ld = ld[s];
        k.gscale = n[s] > 0 ? 1.f / (float)n[s] : 0.f;
        B->probs.push_back(problems[s]);
        B->skels.push_back(k);
    }
    int rc = CT_OK;
    if (hipMalloc(&B->d_skels, count * sizeof(ct::BatchSkel)) != hipSuccess ||
        hipMalloc(&B->d_queue, 2 * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&B->t_dev, 2 * sizeof(int32_t)) != hipSuccess)
        rc = CT_ERR_ALLOC;
    if (rc == CT_OK && hipMemcpy(B->d_skels, B->skels.data(), count * sizeof(ct::BatchSkel),
                                 hipMemcpyHostToDevice) != hipSuccess)
        rc = CT_ERR_DEVICE;
    if (rc == CT_OK && hipMemset(B->d_queue, 0, 2 * sizeof(int32_t)) != hipSuccess) rc = CT_ERR_DEVICE;
    if (rc == CT_OK) rc = batch_build_items(B);
    if (rc != CT_OK) {
        ct_batch_destroy(B);
        return rc;
    }
    *out = B;
    return CT_OK;
}

extern "C" int ct_batch_destroy(ct_batch* B) {
    if (!B) return CT_OK;
    hipDeviceSynchronize();   // eager launches may still read the work list and queue
    batch_drop_graph(B);
    if (B->replayed) hipEventDestroy(B->replayed);
    if (B->capture_stream) hipStreamDestroy(B->capture_stream);
    if (B->d_skels) hipFree(B->d_skels);
    if (B->d_items) hipFree(B->d_items);
    if (B->d_queue) hipFree(B->d_queue);
    if (B->t_dev) hipFree(B->t_dev);
    delete B;
    return CT_OK;
}

extern "C" int ct_batch_set_tuning(ct_batch* B, int32_t split, int32_t workgroups, int32_t persistent) {
    if (!B || !(split == 0 || split == 1 || split == 2 || split == 4) || workgroups < 0) return CT_ERR_INVALID_ARG;
    const bool rebuild = batch_split(B) != (split ? split : 1);
    B->split = split;
    B->workgroups = workgroups;
    B->persistent = persistent ? 1 : 0;
    batch_drop_graph(B);
    return rebuild ? batch_build_items(B) : CT_OK;
}

extern "C" int ct_batch_step(ct_batch* B, int64_t t, const ct_adam* adam, void* stream) {
    if (!B || t < 1 || t > INT32_MAX || !valid_adam(adam)) return CT_ERR_INVALID_ARG;
    return batch_launch(B, adam, (int32_t)t, nullptr, nullptr, (hipStream_t)stream);
}

extern "C" int ct_batch_optimize(ct_batch* B, int64_t t0, int32_t iters, const ct_adam* adam, void* stream) {
    if (!B || t0 < 0 || iters < 0 || t0 + iters > INT32_MAX || !valid_adam(adam)) return CT_ERR_INVALID_ARG;
    if (iters == 0) return CT_OK;
    const bool same = B->gexec && B->g_iters == iters && B->g_split == batch_split(B) &&
                      B->g_wg == batch_workgroups(B) && B->g_pers == B->persistent && B->g_lr == adam->lr &&
                      B->g_b1 == adam->beta1 && B->g_b2 == adam->beta2 && B->g_eps == adam->eps;
    if (!same) {
        batch_drop_graph(B);
        if (!B->capture_stream && hipStreamCreateWithFlags(&B->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return CT_ERR_DEVICE;
        if (hipStreamBeginCapture(B->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return CT_ERR_DEVICE;
        int rc = CT_OK;
        for (int32_t it = 0; it < iters && rc == CT_OK; ++it)
            rc = batch_launch(B, adam, 0, B->t_dev + (it & 1), B->t_dev + ((it + 1) & 1), B->capture_stream);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(B->capture_stream, &g);
        if (rc != CT_OK || ec != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            return rc != CT_OK ? rc : CT_ERR_DEVICE;
        }
        hipGraphExec_t ge = nullptr;
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            return CT_ERR_DEVICE;
        }
        B->graph = g;
        B->gexec = ge;
        B->g_iters = iters;
        B->g_split = batch_split(B);
        B->g_wg = batch_workgroups(B);
        B->g_pers = B->persistent;
        B->g_lr = adam->lr; B->g_b1 = adam->beta1; B->g_b2 = adam->beta2; B->g_eps = adam->eps;
    }
    if (!B->replayed && hipEventCreateWithFlags(&B->replayed, hipEventDisableTiming) != hipSuccess) {
        B->replayed = nullptr;
        return CT_ERR_DEVICE;
    }
    hipLaunchKernelGGL(ct::counter_set_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream, B->t_dev, (int32_t)t0);
    int rc = err_of(hipGetLastError());
    if (rc != CT_OK) return rc;
    rc = err_of(hipGraphLaunch(B->gexec, (hipStream_t)stream));
    if (rc != CT_OK) return rc;
    return err_of(hipEventRecord(B->replayed, (hipStream_t)stream));
}

extern "C" int ct_batch_autotune(ct_batch* B, int32_t* chosen, void* stream) {
    if (!B) return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const ct_adam adam{0.f, 0.9f, 0.999f, 1e-8f, 1.f};   // lr 0: X stays as it is
    const int keep_pers = B->persistent;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CT_ERR_DEVICE;
    float best = 1e30f;
    int best_split = 1, best_wg = 2 * B->n_cu, rc = CT_OK;
    for (int split : {1, 2}) {
        for (int per_cu : {1, 2, 3, 4}) {
            rc = ct_batch_set_tuning(B, split, per_cu * B->n_cu, 1);
            if (rc != CT_OK) break;
            for (int w = 0; w < 2 && rc == CT_OK; ++w) rc = batch_launch(B, &adam, 1, nullptr, nullptr, st);
            hipEventRecord(e0, st);
            for (int r = 0; r < 5 && rc == CT_OK; ++r) rc = batch_launch(B, &adam, 2 + r, nullptr, nullptr, st);
            hipEventRecord(e1, st);
            if (rc != CT_OK) break;
            if (hipEventSynchronize(e1) != hipSuccess) { rc = CT_ERR_DEVICE; break; }
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; best_split = split; best_wg = per_cu * B->n_cu; }
        }
        if (rc != CT_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    for (const auto& k : B->skels) {
        if (k.n == 0) continue;
        const size_t bytes = (size_t)k.ld * (size_t)B->probs[&k - B->skels.data()]->D * sizeof(float);
        hipMemsetAsync(k.M, 0, bytes, st);
        hipMemsetAsync(k.V, 0, bytes, st);
    }
    if (rc != CT_OK) return rc;
    rc = ct_batch_set_tuning(B, best_split, best_wg, keep_pers);
    if (chosen) { chosen[0] = best_split; chosen[1] = best_wg; }
    return rc;
}
