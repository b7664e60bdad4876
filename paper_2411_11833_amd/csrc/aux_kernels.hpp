// Elementwise kernels around the fused step: the uniform initializer and the
// stand-alone Adam update.
#pragma once

#include "ct_tables.hpp"
#include "philox.hpp"

namespace ct {

// One thread per particle: uniform draw inside the initialization box for
// every dimension (stores coalesced along particles), moments zeroed.
__global__ __launch_bounds__(256) void seed_uniform_kernel(const Tables* __restrict__ T, uint32_t k0,
                                                           uint32_t k1, float* __restrict__ X,
                                                           float* __restrict__ M, float* __restrict__ V,
                                                           int64_t n, int64_t ld) {
#pragma clang fp contract(off)
    // lo + (hi - lo) u with one rounding per operation (no fused multiply-add),
    // so that any IEEE single-precision implementation reproduces it bit for bit
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int D = T->D;
    for (int b = 0; 4 * b < D; ++b) {
        uint32_t c[4] = {(uint32_t)i, (uint32_t)b, 0u, 0u};
        philox4x32_10(c, k0, k1);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int d = 4 * b + w;
            if (d < D) {
                const float u = (float)(c[w] >> 8) * 5.9604644775390625e-08f;   // 2^-24
                const float lo = T->lo[d], hi = T->hi[d];
                X[d * ld + i] = lo + (hi - lo) * u;
                if (M) M[d * ld + i] = 0.f;
                if (V) V[d * ld + i] = 0.f;
            }
        }
    }
}

// Placement sampler of compositional initialization (Sec. V): after the
// uniform draw, the placement centre of every step is redrawn uniformly over
// the centres that keep the object's footprint, turned by the drawn yaw psi,
// inside the goal region: on each axis [lo + e, hi - e] with
// e_x = |hx cos psi| + |hy sin psi|, e_y = |hx sin psi| + |hy cos psi|, from
// the same Philox word as the uniform draw of that dimension (the region's
// centre when the interval is empty).  Joint and grasp dimensions keep the
// uniform draw: the grasp box is the Grasp constraint's set, and uniform
// configurations are the starting points of the configuration sampler.
__global__ __launch_bounds__(256) void place_sampler_kernel(const Tables* __restrict__ T, uint32_t k0, uint32_t k1,
                                                            float* __restrict__ X, int64_t n, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < T->K; ++k) {
        const int o = CT_STEP_DIM * k;
        const float psi = X[(int64_t)(o + 20) * ld + i];
        float sn, cs;
        sincosf(psi, &sn, &cs);
        const float hx = T->obj0[k].hx, hy = T->obj0[k].hy;
        const float e[2] = {fabsf(hx * cs) + fabsf(hy * sn), fabsf(hx * sn) + fabsf(hy * cs)};
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            const int d = o + 18 + ax;
            uint32_t c[4] = {(uint32_t)i, (uint32_t)(d / 4), 0u, 0u};
            philox4x32_10(c, k0, k1);
            const float u = (float)(c[d % 4] >> 8) * 5.9604644775390625e-08f;   // 2^-24
            const float a = T->region_lo[ax] + e[ax], b = T->region_hi[ax] - e[ax];
            X[(int64_t)d * ld + i] = b >= a ? a + (b - a) * u : 0.5f * (T->region_lo[ax] + T->region_hi[ax]);
        }
    }
}

// Stand-alone Adam: one thread per particle, so that a particle with a
// non-finite gradient or coordinate is skipped as a whole.
__global__ __launch_bounds__(256) void adam_kernel(int D, float* __restrict__ X, float* __restrict__ M,
                                                   float* __restrict__ V, const float* __restrict__ G,
                                                   const uint8_t* __restrict__ frozen, int64_t n, int64_t ld,
                                                   float lr, float b1, float b2, float eps, float gscale,
                                                   int32_t t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float bc1 = 1.f - powf(b1, (float)t), bc2 = 1.f - powf(b2, (float)t);
    bool fin = true;
    for (int d = 0; d < D; ++d) {
        const float s = G[d * ld + i] + X[d * ld + i];
        fin = fin && __builtin_isfinite(s);
    }
    if (!fin) return;
    for (int d = 0; d < D; ++d) {
        if (frozen && frozen[d]) continue;
        const int64_t a = d * ld + i;
        const float gs = gscale * G[a];
        const float m1 = b1 * M[a] + (1.f - b1) * gs;
        const float v1 = b2 * V[a] + (1.f - b2) * gs * gs;
        X[a] = X[a] - lr * (m1 / bc1) / (sqrtf(v1 / bc2) + eps);
        M[a] = m1;
        V[a] = v1;
    }
}

// Device counter of applied Adam updates, set before a captured loop.
__global__ void counter_set_kernel(int32_t* c, int32_t v) { *c = v; }

// Tolerance of constraint term c (per step: Kin position / rotation at the
// pick and at the place, grasp box, placement, two joint-limit terms, three
// collision terms; then the motion-collision terms, then the self-collision
// terms).
__device__ __forceinline__ float term_eps(const Tables* __restrict__ T, int c) {
    if (T->self_term >= 0 && c >= T->self_term) return T->eps[E_SELF];
    if (c >= CT_TERMS_PER_STEP * T->K) return T->eps[E_MCOLL];
    switch (c % CT_TERMS_PER_STEP) {
        case T_PICK_POS: case T_PLACE_POS: return T->eps[E_KPOS];
        case T_PICK_ROT: case T_PLACE_ROT: return T->eps[E_KROT];
        case T_GRASP: return T->eps[E_GRASP];
        case T_PLACE: return T->eps[E_PLACE];
        case T_JLIM_G: case T_JLIM_P: return T->eps[E_JLIM];
        default: return T->eps[E_COLL];
    }
}

// Weight lambda of term c of Eq. (2), in the term order of term_eps followed
// by the soft costs (goal, TrajLength).
__device__ __forceinline__ float term_weight(const Tables* __restrict__ T, int c) {
    if (c == T->goal_term) return T->w[W_GOAL];
    if (c == T->traj_term) return T->w[W_TRAJ];
    if (T->self_term >= 0 && c >= T->self_term) return T->w[W_SELF];
    if (c >= CT_TERMS_PER_STEP * T->K) return T->w[W_MCOLL];
    switch (c % CT_TERMS_PER_STEP) {
        case T_PICK_POS: case T_PLACE_POS: return T->w[W_KPOS];
        case T_PICK_ROT: case T_PLACE_ROT: return T->w[W_KROT];
        case T_GRASP: return T->w[W_GRASP];
        case T_PLACE: return T->w[W_PLACE];
        case T_JLIM_G: case T_JLIM_P: return T->w[W_JLIM];
        default: return T->w[W_COLL];
    }
}

// Multiplier update of the augmented-Lagrangian mode for every particle i < n
// and term c, arrays [n_terms][ld]: a constraint J_c <= eps_c is the
// inequality g_c = J_c - eps_c <= 0, so mu_c <- max(0, mu_c + rho g_c) (kept
// when J_c is not finite) and the term's weight becomes W_c = lambda_c + mu_c;
// a soft cost keeps W_c = lambda_c.
__global__ __launch_bounds__(256) void al_update_kernel(const Tables* __restrict__ T, const float* __restrict__ terms,
                                                        int64_t n, int64_t ld, float rho, float* __restrict__ mu,
                                                        float* __restrict__ W) {
    const int64_t total = (int64_t)T->n_terms * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
        const int c = (int)(idx / n);
        const int64_t a = (int64_t)c * ld + (idx - (int64_t)c * n);
        const float lam = term_weight(T, c);
        if (c < T->n_constraint) {
            const float J = terms[a];
            float m = mu[a];
            if (__builtin_isfinite(J)) m = fmaxf(0.f, fmaf(rho, J - term_eps(T, c), m));
            mu[a] = m;
            W[a] = lam + m;
        } else {
            W[a] = lam;
        }
    }
}

// Weights of the PHR augmented Lagrangian at the particles' current terms:
// for the inequality g_c = J_c - eps_c <= 0 with multiplier mu_c >= 0 and
// penalty rho, L = sum_c lambda_c J_c + (1 / 2 rho) sum_c (max(0, mu_c +
// rho g_c)^2 - mu_c^2) has dL/dx = sum_c (lambda_c + max(0, mu_c + rho g_c))
// dJ_c/dx, so W_c = lambda_c + max(0, mu_c + rho (J_c - eps_c)) (lambda_c +
// mu_c when J_c is not finite); soft costs keep lambda_c.  mu is not changed.
__global__ __launch_bounds__(256) void al_weights_kernel(const Tables* __restrict__ T, const float* __restrict__ terms,
                                                         int64_t n, int64_t ld, float rho,
                                                         const float* __restrict__ mu, float* __restrict__ W) {
    const int64_t total = (int64_t)T->n_terms * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
        const int c = (int)(idx / n);
        const int64_t a = (int64_t)c * ld + (idx - (int64_t)c * n);
        const float lam = term_weight(T, c);
        if (c < T->n_constraint) {
            const float J = terms[a];
            const float m = mu[a];
            W[a] = lam + (__builtin_isfinite(J) ? fmaxf(0.f, fmaf(rho, J - term_eps(T, c), m)) : m);
        } else {
            W[a] = lam;
        }
    }
}

// Plan-skeleton feasibility, Eq. (5): one workgroup per constraint term
// counts the particles with J_c <= eps_c (reads coalesced along particles; a
// NaN term never counts), fixed-order tree reduction.
__global__ __launch_bounds__(256) void feas_count_kernel(const Tables* __restrict__ T, const float* __restrict__ terms,
                                                         int64_t n, int64_t ld, int32_t* __restrict__ counts) {
    __shared__ int red[256];
    const int c = blockIdx.x;
    const float e = term_eps(T, c);
    int cnt = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) cnt += terms[(int64_t)c * ld + i] <= e ? 1 : 0;
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[c] = red[0];
}

// H = (1 / |con|) sum_c h_c, h_c = counts[c] if positive else the penalty;
// summed in constraint order by one lane (integers and the penalty are exact
// in FP32 up to 2^24, so only the division rounds).
__global__ void feas_h_kernel(const int32_t* __restrict__ counts, int nc, float penalty, float* __restrict__ H) {
    if (threadIdx.x != 0) return;
    float s = 0.f;
    for (int c = 0; c < nc; ++c) s += counts[c] > 0 ? (float)counts[c] : penalty;
    *H = nc > 0 ? s / (float)nc : 0.f;
}

// Eq. (3) restricted to each pick-place step: step_mask[k][i] = 1 iff every
// constraint term of step k (its CT_TERMS_PER_STEP terms) is within its
// tolerance; count[i] = how many of the particle's constraint terms are (a
// NaN term never is).  One thread per particle, terms as ct_cost writes them.
__global__ __launch_bounds__(256) void step_mask_kernel(const Tables* __restrict__ T,
                                                        const float* __restrict__ terms, int64_t n, int64_t ld,
                                                        uint8_t* __restrict__ step_mask, int64_t ld_mask,
                                                        int32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int total = 0;
    for (int k = 0; k < T->K; ++k) {
        int all = 1;
        for (int j = 0; j < CT_TERMS_PER_STEP; ++j) {
            const int c = CT_TERMS_PER_STEP * k + j;
            const int ok = terms[(int64_t)c * ld + i] <= term_eps(T, c) ? 1 : 0;
            all &= ok;
            total += ok;
        }
        if (step_mask) step_mask[(int64_t)k * ld_mask + i] = (uint8_t)all;
    }
    for (int c = CT_TERMS_PER_STEP * T->K; c < T->n_constraint; ++c)
        total += terms[(int64_t)c * ld + i] <= term_eps(T, c) ? 1 : 0;
    if (count) count[i] = total;
}

// Indices of the set entries of a mask, in index order (one workgroup of
// 1024 lanes; each lane scans a contiguous chunk, then a block-wide prefix
// sum of the chunk counts places the chunks).
__global__ __launch_bounds__(1024) void compact_kernel(const uint8_t* __restrict__ mask, int64_t n,
                                                       int32_t* __restrict__ idx, int32_t* __restrict__ count) {
    __shared__ int32_t pre[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t a = tid * chunk, b = a + chunk < n ? a + chunk : n;
    int32_t c = 0;
    for (int64_t i = a; i < b; ++i) c += mask[i] ? 1 : 0;
    pre[tid] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan
        const int32_t v = tid >= o ? pre[tid - o] : 0;
        __syncthreads();
        pre[tid] += v;
        __syncthreads();
    }
    int32_t w = pre[tid] - c;
    for (int64_t i = a; i < b; ++i)
        if (mask[i]) idx[w++] = (int32_t)i;
    if (tid == 1023) *count = pre[1023];
}

// X[row0 + r][i] = Xs[r][j(i)] for r < rows, i < n, with j(i) = idx[i mod c]
// when c = *count > 0, else i mod n_src; M and V of those rows zeroed.
__global__ __launch_bounds__(256) void gather_block_kernel(const float* __restrict__ Xs, int64_t lds, int rows,
                                                           const int32_t* __restrict__ idx,
                                                           const int32_t* __restrict__ count, int64_t n_src,
                                                           float* __restrict__ X, float* __restrict__ M,
                                                           float* __restrict__ V, int64_t ld, int row0, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = count ? *count : 0;
    const int64_t j = c > 0 ? (int64_t)idx[i % c] : i % n_src;
    for (int r = 0; r < rows; ++r) {
        X[(int64_t)(row0 + r) * ld + i] = Xs[(int64_t)r * lds + j];
        if (M) M[(int64_t)(row0 + r) * ld + i] = 0.f;
        if (V) V[(int64_t)(row0 + r) * ld + i] = 0.f;
    }
}

}  // namespace ct

