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
// collision terms; then the motion-collision terms).
__device__ __forceinline__ float term_eps(const Tables* __restrict__ T, int c) {
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

}  // namespace ct

