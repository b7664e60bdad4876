// Kernels of the learned seed proposer: a multilayer perceptron whose matrix
// products run on the CDNA4 matrix cores in BF16 with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16), with GELU, Gaussian input noise, nearest-draw
// (IMLE) selection, the squared-error gradient, bias sums and Adam around them.
//
// Every product is written C = A * B^T with both operands K-contiguous BF16:
//   forward   Z_l   = H_{l-1} * W_l^T        (A = H [rows][in],  B = W   [out][in])
//   backward  dH    = dZ_l * W_l             (A = dZ [rows][out], B = W^T [in][out])
//   weights   dW_l  = dZ_l^T * H_{l-1}       (A = dZ^T [out][rows], B = H^T [in][rows])
// so the epilogues store activations and gradients in both orientations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace ct {
namespace mlp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));   // 16 bytes moved as one value
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// two floats -> packed bfloat16 bits (first in the low half), round to
// nearest, ties to even: one v_cvt_pk_bf16_f32
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t{a, b}), bf16x2_t));
}

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Phi(x), the standard normal CDF, as erfc(u) / 2 at u = -x / sqrt 2, with
// erfc(u) = t exp(-u^2 + P(t)), t = 1 / (1 + u / 2) for u >= 0 and P the
// degree-9 Chebyshev interpolant that norm_cdf_fit.py derives (relative error
// of erfc about 1e-7).  Branch-free, one reciprocal and one exponential, and
// accurate relative to Phi in the lower tail, where 1 + erf(x / sqrt 2)
// cancels.  Used by the backward epilogue's GELU derivative.
__device__ __forceinline__ float norm_cdf(float x) {
    const float a = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(a, 0.35355339059327376f, 1.f));   // a / sqrt 2 = u
    float p = 0.17087277768357076f;
    p = fmaf(p, t, -0.82215223447300323f);
    p = fmaf(p, t, 1.4885158894086188f);
    p = fmaf(p, t, -1.1352040006480935f);
    p = fmaf(p, t, 0.27886808472408969f);
    p = fmaf(p, t, -0.18628806181001004f);
    p = fmaf(p, t, 0.096784189536313278f);
    p = fmaf(p, t, 0.37409195971065135f);
    p = fmaf(p, t, 1.0000236801583804f);
    p = fmaf(p, t, -1.26551222514161f);
    const float y = fmaf(-0.5f * a, a, p);   // -u^2 + P(t)
    const float q = t * __builtin_amdgcn_exp2f(fmaf(y, 1.4426950408889634f, -1.f));   // erfc(|u|) / 2
    return x >= 0.f ? 1.f - q : q;
}

// GELU of the forward epilogues, x Phi(x), with Phi on [-8, 8] as 512 cubic
// pieces: the Hermite interpolant of Phi and phi at the nodes -8 + k / 32,
// held per piece as coefficients c0..c3 of its polynomial in the fraction f
// of the way across it, built once per handle in double precision
// (gelu_table_kernel) and read from an LDS copy.  Interpolation error below
// 2e-9 (h^4 max|Phi^(4)| / 384); outside [-8, 8] Phi is 0 or 1 to FP32
// precision and the end pieces give exactly that.  Rounded to BF16, x Phi(x)
// this way differs from the exact GELU on about 7e-6 of FP32 inputs in
// [-8, 8] (the erf form: 3e-3), at 9 VALU instructions and one LDS read.
constexpr int GELU_PIECES = 512;
constexpr int GELU_TAB_BYTES = GELU_PIECES * 16;

__device__ __forceinline__ float gelu_tab(const f32x4_t* __restrict__ tab, float x) {
    const float u = __builtin_amdgcn_fmed3f(fmaf(x, 32.f, 256.f), 0.f, 511.99994f);
    const f32x4_t c = tab[(int)u];
    const float f = __builtin_amdgcn_fractf(u);
    return x * fmaf(fmaf(fmaf(c[3], f, c[2]), f, c[1]), f, c[0]);
}

__global__ __launch_bounds__(256) void gelu_table_kernel(f32x4_t* __restrict__ tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= GELU_PIECES) return;
    const double h = 1.0 / 32, z0 = -8.0 + k * h, z1 = z0 + h;
    const double p0 = 0.5 * erfc(-z0 * 0.70710678118654752), p1 = 0.5 * erfc(-z1 * 0.70710678118654752);
    const double d0 = h * 0.39894228040143268 * exp(-0.5 * z0 * z0);
    const double d1 = h * 0.39894228040143268 * exp(-0.5 * z1 * z1);
    tab[k] = f32x4_t{(float)p0, (float)d0, (float)(3.0 * (p1 - p0) - 2.0 * d0 - d1), (float)(2.0 * (p0 - p1) + d0 + d1)};
}

// d/dx [x Phi(x)] = Phi(x) + x phi(x)
__device__ __forceinline__ float gelu_grad(float x) {
    return fmaf(x * 0.39894228040143268f, __builtin_amdgcn_exp2f(-0.72134752044448170f * x * x), norm_cdf(x));
}

// Bijection from the launch index to a tile index that gives each of the 8
// XCDs (workgroups are dealt to them round-robin) a contiguous range of
// tiles, so that the tiles sharing rows of A (consecutive in N) share an L2.
__device__ __forceinline__ int xcd_swizzle(int b, int G) {
    constexpr int NX = 8;
    const int x = b % NX, q = G / NX, rem = G % NX;
    return x * q + (x < rem ? x : rem) + b / NX;
}

// Four standard normals from one Philox block: Box-Muller on the word pairs
// (w0, w1) and (w2, w3), u1 = 1 - (w >> 8) 2^-24 in (0, 1], u2 = (w >> 8) 2^-24.
__device__ __forceinline__ void normal4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t k0, uint32_t k1,
                                        float z[4]) {
    uint32_t c[4] = {c0, c1, c2, 0u};
    philox4x32_10(c, k0, k1);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float u1 = 1.f - (float)(c[2 * p] >> 8) * 5.9604644775390625e-08f;
        const float u2 = (float)(c[2 * p + 1] >> 8) * 5.9604644775390625e-08f;
        const float rad = sqrtf(-2.f * logf(u1));
        float s, co;
        sincospif(2.f * u2, &s, &co);
        z[2 * p] = rad * co;
        z[2 * p + 1] = rad * s;
    }
}

// ---------------------------------------------------------------------------
// C = A * B^T on the matrix cores

enum Epi { EPI_HID_TRAIN = 0, EPI_HID_INFER = 1, EPI_OUT = 2, EPI_BWD = 3, EPI_DW = 4 };

struct GemmArgs {
    const uint16_t* A;
    int64_t lda;   // [M][K] BF16, K contiguous
    const uint16_t* B;
    int64_t ldb;   // [N][K] BF16, K contiguous
    int M, N, K;   // K % (32 * ksplit) == 0
    int ksplit;    // K chunks, one workgroup each (EPI_DW only)
    const float* bias;   // [N]  (HID_*, OUT)
    float* F;            // HID_TRAIN: Z [M][N]; OUT: Y [M][N]; DW: partial [ksplit][M][N] or dW
    int64_t ldf, fsplit;
    const float* Zin;    // BWD: pre-activation of the layer the gradient flows into, [M][N]
    int64_t ldzin;
    uint16_t* Hb;        // HID_*: H = bf16(gelu(Z)); BWD: D = bf16(dH * gelu'(Zin));  [M][N]
    int64_t ldh;
    uint16_t* Ht;        // the same values transposed, [N][ldht] (HID_TRAIN, BWD)
    int64_t ldht;
    const f32x4_t* gelu_tab;   // GELU_PIECES pieces (HID_*)
};

constexpr int GT = 32;    // workgroup tile (M and N) of the split-K weight-gradient products (K slices 64 deep)
constexpr int GT_SHALLOW = 64;   // the same where a K chunk is not a multiple of 64 (slices 32 deep)
constexpr int GK = 32;    // K per MFMA (and the granularity of K and of split-K chunks)
constexpr int GPAD = 8;   // LDS row padding (BF16 elements)

// Epilogue of a TM x TN output tile computed by WM x WN waves (NT = 64 WM WN
// threads), each wave owning FI x FJ accumulator tiles of 16 x 16.  Values
// (bias, GELU or its derivative) are formed in registers and FP32 outputs
// stored from there; BF16 outputs are staged in LDS (`stage`, TM x (TN + 8)
// elements, free once the main loop is done) and leave as 16-byte chunks of
// rows; the training epilogues' transposed copy leaves from registers (a
// lane holds 4 consecutive rows of one column: 8 bytes of the transpose).
template <int EPI, int TM, int TN, int FI, int FJ, int WM = 2, int WN = 2>
__device__ __forceinline__ void tile_epilogue(const GemmArgs& g, const f32x4_t (&acc)[FI][FJ], int m0, int n0,
                                              int split, uint16_t* __restrict__ stage, const f32x4_t* tab) {
    constexpr bool BF = EPI == EPI_HID_TRAIN || EPI == EPI_HID_INFER || EPI == EPI_BWD;
    constexpr bool TR = EPI == EPI_HID_TRAIN || EPI == EPI_BWD;
    constexpr int LDT = TN + 8;
    constexpr int NT = 64 * WM * WN;
    static_assert(FI * 16 * WM == TM && FJ * 16 * WN == TN, "wave tiles must cover the tile");
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w / WN, wn = w % WN;
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
        const int cl = wn * (TN / WN) + j * 16 + (lane & 15), n = n0 + cl;
        float bias = 0.f;
        if constexpr (EPI == EPI_HID_TRAIN || EPI == EPI_HID_INFER || EPI == EPI_OUT)
            if (n < g.N) bias = g.bias[n];
#pragma unroll
        for (int i = 0; i < FI; ++i) {
            const int rl0 = wm * (TM / WM) + i * 16 + (lane >> 4) * 4;
            uint16_t h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rl = rl0 + r, m = m0 + rl;
                const bool ok = m < g.M && n < g.N;
                const float v = acc[i][j][r];
                h[r] = 0;
                if constexpr (EPI == EPI_HID_TRAIN || EPI == EPI_HID_INFER) {
                    const float z = v + bias;
                    if (EPI == EPI_HID_TRAIN && ok) g.F[(int64_t)m * g.ldf + n] = z;
                    if (ok) h[r] = to_bf16(gelu_tab(tab, z));
                    stage[rl * LDT + cl] = h[r];
                } else if constexpr (EPI == EPI_BWD) {
                    if (ok) h[r] = to_bf16(v * gelu_grad(g.Zin[(int64_t)m * g.ldzin + n]));
                    stage[rl * LDT + cl] = h[r];
                } else if constexpr (EPI == EPI_OUT) {
                    if (ok) g.F[(int64_t)m * g.ldf + n] = v + bias;
                } else {
                    if (ok) g.F[(int64_t)split * g.fsplit + (int64_t)m * g.ldf + n] = v;
                }
            }
            if constexpr (TR) {
                // the transposed copy straight from registers: this lane's 4
                // rows are 4 consecutive entries of row n of the transpose
                const int m = m0 + rl0;
                if (n < g.N && m < g.M) {
                    uint16_t* dst = g.Ht + (int64_t)n * g.ldht + m;
                    if (m + 4 <= g.M) {
                        *(uint2*)dst = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                                  (uint32_t)h[2] | ((uint32_t)h[3] << 16));
                    } else {
                        for (int r = 0; r < 4 && m + r < g.M; ++r) dst[r] = h[r];
                    }
                }
            }
        }
    }
    if constexpr (BF) {
        __syncthreads();
        constexpr int CH = TN / 8;   // 16-byte chunks of a row
        for (int c = tid; c < TM * CH; c += NT) {
            const int rl = c / CH, cl = (c - rl * CH) * 8, m = m0 + rl, n = n0 + cl;
            if (m >= g.M || n >= g.N) continue;
            uint16_t* dst = g.Hb + (int64_t)m * g.ldh + n;
            if (n + 8 <= g.N) {
                *(u32x4_t*)dst = *(const u32x4_t*)(stage + rl * LDT + cl);
            } else {
                for (int q = 0; n + q < g.N; ++q) dst[q] = stage[rl * LDT + cl + q];
            }
        }
    }
}

// C = A * B^T over a TILE x TILE workgroup tile (TILE = 64; split-K over
// ksplit workgroups per tile): the weight-gradient products, whose K (the
// rows of a batch) is split into chunks.  256 threads = 4 waves in a 2 x 2
// arrangement, each wave a (TILE/2) x (TILE/2) block of FI x FI MFMA
// 16x16x32 tiles.  Operand fragments: lane l holds row (l % 16) and K
// elements 8 (l / 16) .. 8 (l / 16) + 7 of its 16 x 32 A and B blocks;
// accumulator element r of lane l is C[4 (l / 16) + r][l % 16].  K is staged
// BK (32 or 64) deep through two LDS buffers: the global loads of the next
// slice are in flight while this slice's products run, and one barrier per
// slice orders the buffers.  Tile order is XCD-aware (tiles sharing rows of
// A share an L2).
template <int TILE, int BK>
union GemmSmem {
    struct {
        uint16_t A[2][TILE][BK + GPAD];
        uint16_t B[2][TILE][BK + GPAD];
    } k;
    uint16_t stage[TILE * (TILE + 8)];
};

template <int EPI, int TILE, int BK>
__device__ __forceinline__ void gemm_nt_tile(const GemmArgs& g, int block, int n_blocks) {
    constexpr int FI = TILE / 32;           // MFMA tiles per wave and dimension
    constexpr int CPR = BK / 8;             // 16-byte chunks per row of a slice
    constexpr int RPP = 256 / CPR;          // rows one pass of the workgroup loads
    constexpr int H = TILE / RPP;           // chunks per thread and operand per slice
    constexpr int KH = BK / 32;             // MFMA depths per slice
    __shared__ __attribute__((aligned(16))) GemmSmem<TILE, BK> sm;
    auto& As = sm.k.A;
    auto& Bs = sm.k.B;
    const int tiles_n = (g.N + TILE - 1) / TILE;
    int bid = xcd_swizzle(block, n_blocks);
    const int split = bid % g.ksplit;
    bid /= g.ksplit;
    const int m0 = (bid / tiles_n) * TILE, n0 = (bid % tiles_n) * TILE;
    const int kc = g.K / g.ksplit, kb = split * kc;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int lr = tid / CPR, lk = (tid % CPR) * 8;   // rows lr + RPP h
    bool aok[H], bok[H];
    const uint16_t* pa[H];
    const uint16_t* pb[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int ra = m0 + lr + RPP * h, rb = n0 + lr + RPP * h;
        aok[h] = ra < g.M;
        bok[h] = rb < g.N;
        pa[h] = g.A + (int64_t)(aok[h] ? ra : 0) * g.lda + kb + lk;
        pb[h] = g.B + (int64_t)(bok[h] ? rb : 0) * g.ldb + kb + lk;
    }
    f32x4_t acc[FI][FI];
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FI; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const u32x4_t z4 = {0u, 0u, 0u, 0u};
    u32x4_t ra[H], rb[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        ra[h] = aok[h] ? *(const u32x4_t*)(pa[h]) : z4;
        rb[h] = bok[h] ? *(const u32x4_t*)(pb[h]) : z4;
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
        *(u32x4_t*)&As[0][lr + RPP * h][lk] = ra[h];
        *(u32x4_t*)&Bs[0][lr + RPP * h][lk] = rb[h];
    }
    __syncthreads();
    const int steps = kc / BK;
    for (int st = 0; st < steps; ++st) {
        const int cur = st & 1;
        const bool more = st + 1 < steps;
        if (more) {
            const int k1 = (st + 1) * BK;
#pragma unroll
            for (int h = 0; h < H; ++h) {
                ra[h] = aok[h] ? *(const u32x4_t*)(pa[h] + k1) : z4;
                rb[h] = bok[h] ? *(const u32x4_t*)(pb[h] + k1) : z4;
            }
        }
#pragma unroll
        for (int kh = 0; kh < KH; ++kh) {
            bf16x8_t af[FI], bf[FI];
#pragma unroll
            for (int i = 0; i < FI; ++i)
                af[i] = __builtin_bit_cast(bf16x8_t, *(const u32x4_t*)&As[cur][wm * (TILE / 2) + i * 16 + (lane & 15)]
                                                                      [kh * 32 + (lane >> 4) * 8]);
#pragma unroll
            for (int j = 0; j < FI; ++j)
                bf[j] = __builtin_bit_cast(bf16x8_t, *(const u32x4_t*)&Bs[cur][wn * (TILE / 2) + j * 16 + (lane & 15)]
                                                                      [kh * 32 + (lane >> 4) * 8]);
#pragma unroll
            for (int i = 0; i < FI; ++i)
#pragma unroll
                for (int j = 0; j < FI; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
            // the other buffer was last read in step st - 1, which every wave
            // finished before the barrier at the end of that step
#pragma unroll
            for (int h = 0; h < H; ++h) {
                *(u32x4_t*)&As[cur ^ 1][lr + RPP * h][lk] = ra[h];
                *(u32x4_t*)&Bs[cur ^ 1][lr + RPP * h][lk] = rb[h];
            }
        }
        __syncthreads();
    }
    // the loop ends with a barrier after the last fragment reads: the LDS is the stage now
    tile_epilogue<EPI, TILE, TILE, FI, FI>(g, acc, m0, n0, split, sm.stage, nullptr);
}

template <int EPI, int TILE, int BK>
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g) {
    gemm_nt_tile<EPI, TILE, BK>(g, (int)blockIdx.x, (int)gridDim.x);
}

// Every layer's weight-gradient product of a backward pass in one launch
// (they are independent once the backward products are done): block b runs
// tile b - bstart[l] of layer l.
constexpr int MAX_LAYERS = 9;
struct DwLayers {
    int L;
    int bstart[MAX_LAYERS + 1];   // prefix sums of tiles * ksplit
    GemmArgs g[MAX_LAYERS];
};

template <int BK>
__global__ __launch_bounds__(256) void gemm_dw_layers_kernel(DwLayers a) {
    const int b = (int)blockIdx.x;
    int l = 0;
    while (b >= a.bstart[l + 1]) ++l;
    gemm_nt_tile<EPI_DW, GT, BK>(a.g[l], b - a.bstart[l], a.bstart[l + 1] - a.bstart[l]);
}

// ---------------------------------------------------------------------------
// Pipelined C = A * B^T.  K is staged 32 deep through a ring of S slices in
// LDS that the operands reach by direct global-to-LDS loads
// (global_load_lds_dwordx4: each wave instruction fills 1 KB of LDS, lane l
// the 16 bytes at l * 16), so S - 1 slices are in flight while one is
// multiplied and no registers hold data in transit.  A slice of an operand
// with R rows is R x 32 BF16 = R rows of four 16-byte chunks; chunk c of row
// r sits in slot c ^ sw(r), sw(r) = ((r >> 1) & 3) ^ ((r >> 3) & 1), so that
// any 8 consecutive rows of one chunk column (and any 16) spread over
// distinct 16-byte bank groups: fragment reads are free of bank conflicts.  Rows past M (or N) load
// row M - 1 (N - 1) instead; they only reach outputs that are not stored.
//
// Order per slice s (with the next slice s + 1): wait until this wave's
// loads of s + 1 have landed and its LDS reads are done, barrier (every
// wave's loads of s + 1 are visible and every wave holds the fragments of s
// in registers), issue the loads of slice s + S into the slot of s, read the
// fragments of s + 1, then the MFMAs of s (while those reads return).
// WM x WN waves of (TM / WM) x (TN / WN) outputs each.

// wait until at most n of this wave's vector-memory loads are outstanding
// and all of its LDS reads have returned (n wave-uniform, 0 <= n <= 15)
__device__ __forceinline__ void vm_lds_wait(int n) {
    // s_waitcnt immediate: vmcnt in bits 3:0, lgkmcnt 11:8 (0), expcnt 6:4 left at its maximum
    switch (n) {
#define CT_VMW(k) case k: __builtin_amdgcn_s_waitcnt(0x0070 | k); break;
        CT_VMW(1) CT_VMW(2) CT_VMW(3) CT_VMW(4) CT_VMW(5) CT_VMW(6) CT_VMW(7) CT_VMW(8)
        CT_VMW(9) CT_VMW(10) CT_VMW(11) CT_VMW(12) CT_VMW(13) CT_VMW(14) CT_VMW(15)
#undef CT_VMW
        default: __builtin_amdgcn_s_waitcnt(0x0070); break;
    }
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

template <int TM, int TN, int WM, int WN, int S>
struct PipeCfg {
    static constexpr int NT = 64 * WM * WN;       // threads
    static constexpr int FI = TM / WM / 16, FJ = TN / WN / 16;
    static constexpr int SA = TM * 32, SB = TN * 32;   // BF16 elements of a slice of A, of B
    static constexpr int IA = TM / 16, IB = TN / 16;   // wave instructions that load them (64 chunks each)
    static constexpr int IW = (IA + IB) / (WM * WN);   // per wave and slice
    static constexpr int RING = S * (SA + SB);
    static constexpr int STAGE = TM * (TN + 8);
    static constexpr int MAIN = RING > STAGE ? RING : STAGE;   // BF16 elements; the GELU table follows
    static constexpr int SMEM = MAIN + GELU_TAB_BYTES / 2;
    static_assert(FI * 16 * WM == TM && FJ * 16 * WN == TN, "wave tiles must cover the tile");
    static_assert((IA + IB) % (WM * WN) == 0, "every wave loads the same number of chunks");
    static_assert(IW * (S - 2) <= 15, "loads in flight per wave must fit the wait immediate");
};

// Epilogue straight from the accumulators of the transposed products (SWAP
// below): lane l holds 4 consecutive columns 4 (l / 16) .. + 3 of row l % 16
// of each 16 x 16 block, bias already in them.  Hidden layers store
// bf16(gelu(z)) as 8-byte groups of 4, the output layer FP32 as 16-byte
// groups (where its rows are 16-byte aligned).
template <int EPI, int TM, int TN, int FI, int FJ, int WM, int WN>
__device__ __forceinline__ void reg_epilogue(const GemmArgs& g, const f32x4_t (&acc)[FI][FJ], int m0, int n0,
                                             const f32x4_t* tab) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w / WN, wn = w % WN;
    const bool vec_out = (g.ldf & 3) == 0;
    // whole 16 x 16 blocks inside the output take the unguarded path (a
    // wave-uniform test); blocks on the ragged edges check every element
    const int mw = m0 + wm * (TM / WM), nw = n0 + wn * (TN / WN);
#pragma unroll
    for (int i = 0; i < FI; ++i) {
        const int m = mw + i * 16 + (lane & 15);
        const bool rows_in = mw + i * 16 + 16 <= g.M;
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
            const int n = nw + j * 16 + 4 * (lane >> 4);
            const bool inside = rows_in && nw + j * 16 + 16 <= g.N;
            if constexpr (EPI == EPI_HID_INFER) {
                const uint2 h = make_uint2(pack_bf16(gelu_tab(tab, acc[i][j][0]), gelu_tab(tab, acc[i][j][1])),
                                           pack_bf16(gelu_tab(tab, acc[i][j][2]), gelu_tab(tab, acc[i][j][3])));
                uint16_t* dst = g.Hb + (int64_t)m * g.ldh + n;
                if (inside) {
                    *(uint2*)dst = h;
                } else if (m < g.M) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (n + r < g.N) dst[r] = (uint16_t)((r < 2 ? h.x : h.y) >> (16 * (r & 1)));
                }
            } else {
                float* dst = g.F + (int64_t)m * g.ldf + n;
                if (inside && vec_out) {
                    *(f32x4_t*)dst = acc[i][j];
                } else if (m < g.M) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (n + r < g.N) dst[r] = acc[i][j][r];
                }
            }
        }
    }
}

template <int EPI, int TM, int TN, int WM, int WN, int S>
__global__ __launch_bounds__(64 * WM * WN) void gemm_pipe_kernel(GemmArgs g) {
    using C = PipeCfg<TM, TN, WM, WN, S>;
    constexpr int FI = C::FI, FJ = C::FJ, IW = C::IW;
    // Inference and output products run the MFMA with the operands swapped,
    // accumulating the transpose of each 16 x 16 block, so that a lane ends
    // up with 4 consecutive columns of one row (stored from registers); the
    // training epilogue stages through LDS for its transposed copy instead.
    constexpr bool SWAP = EPI == EPI_HID_INFER || EPI == EPI_OUT;
    static_assert(S >= 3, "the ring holds the slice being read, the next one and the one being loaded");
    __shared__ __attribute__((aligned(1024))) uint16_t sm[C::SMEM];
    const int tiles_n = (g.N + TN - 1) / TN;
    const int bid = xcd_swizzle((int)blockIdx.x, (int)gridDim.x);
    const int m0 = (bid / tiles_n) * TM, n0 = (bid % tiles_n) * TN;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / WN, wn = w % WN;
    // this wave's loads: instructions q = w IW .. w IW + IW - 1 of the slice,
    // the first IA of A, the rest of B; lane l of instruction q fills chunk
    // position 64 q' + l of its operand (q' = q, or q - IA for B)
    const uint16_t* src[IW];
    int dst[IW];
#pragma unroll
    for (int h = 0; h < IW; ++h) {
        const int q = w * IW + h;
        const bool load_a = q < C::IA;
        const int qq = load_a ? q : q - C::IA;
        const int p = qq * 64 + lane, r = p >> 2, c = (p & 3) ^ ((r >> 1) & 3) ^ ((r >> 3) & 1);
        const int row = load_a ? min(m0 + r, g.M - 1) : min(n0 + r, g.N - 1);
        src[h] = (load_a ? g.A + (int64_t)row * g.lda : g.B + (int64_t)row * g.ldb) + c * 8;
        dst[h] = (load_a ? 0 : C::SA) + qq * 512;   // element offset in a ring slot
    }
    auto issue = [&](int s) {
        uint16_t* slot = sm + (s % S) * (C::SA + C::SB);
#pragma unroll
        for (int h = 0; h < IW; ++h)
            __builtin_amdgcn_global_load_lds((const void*)(src[h] + s * 32), (lds_ptr_t)(slot + dst[h]), 16, 0, 0);
    };
    // wait for this wave's loads of slice s (the loads of up to S - 2 later
    // slices stay in flight) and for its LDS reads, then a barrier: every
    // wave's loads of s have landed and every wave holds the fragments it
    // read before.  The empty asm statements keep the compiler from moving
    // LDS accesses across the barrier (it emits no wait of its own).
    const int nk = g.K / 32;
    auto land = [&](int s) {
        vm_lds_wait(min(nk - 1 - s, S - 2) * IW);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    // fragment reads: lane l takes row l % 16 of a 16-row block, chunk l / 16
    const int frag = (lane & 15) * 32 + 8 * ((lane >> 4) ^ ((lane >> 1) & 3) ^ ((lane >> 3) & 1));
    auto read = [&](int s, bf16x8_t (&af)[FI], bf16x8_t (&bf)[FJ]) {
        const uint16_t* As = sm + (s % S) * (C::SA + C::SB);
        const uint16_t* Bs = As + C::SA;
#pragma unroll
        for (int i = 0; i < FI; ++i)
            af[i] = __builtin_bit_cast(bf16x8_t, *(const u32x4_t*)(As + (wm * (TM / WM) + i * 16) * 32 + frag));
#pragma unroll
        for (int j = 0; j < FJ; ++j)
            bf[j] = __builtin_bit_cast(bf16x8_t, *(const u32x4_t*)(Bs + (wn * (TN / WN) + j * 16) * 32 + frag));
    };
    f32x4_t acc[FI][FJ];
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
        f32x4_t b0 = {0.f, 0.f, 0.f, 0.f};
        if constexpr (SWAP) {   // the bias rides in the accumulators
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = n0 + wn * (TN / WN) + j * 16 + 4 * (lane >> 4) + r;
                b0[r] = n < g.N ? g.bias[n] : 0.f;
            }
        }
#pragma unroll
        for (int i = 0; i < FI; ++i) acc[i][j] = b0;
    }
    // the GELU table (hidden layers): 8 KB by direct loads ahead of the
    // ring's, so every wait for a slice covers it too
    constexpr bool GELU = EPI == EPI_HID_TRAIN || EPI == EPI_HID_INFER;
    f32x4_t* tab = (f32x4_t*)(sm + C::MAIN);
    if constexpr (GELU) {
        for (int q = w; q < GELU_PIECES / 64; q += WM * WN)
            __builtin_amdgcn_global_load_lds((const void*)(g.gelu_tab + q * 64 + lane), (lds_ptr_t)(tab + q * 64), 16,
                                             0, 0);
    }
#pragma unroll
    for (int s = 0; s < S - 1; ++s)
        if (s < nk) issue(s);
    // slice s: (if there is a next slice) land it, refill the ring and read
    // its fragments, then multiply slice s -- the next fragments arrive
    // while these MFMAs run
    // (after the last slice the reads fetch a stale slot, unused)
    auto step = [&](int s, bf16x8_t (&af)[FI], bf16x8_t (&bf)[FJ], bf16x8_t (&an)[FI], bf16x8_t (&bn)[FJ]) {
        if (s + 1 < nk) {
            land(s + 1);
            if (s + S < nk) issue(s + S);
        }
        read(s + 1, an, bn);
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
            for (int j = 0; j < FJ; ++j)
                acc[i][j] = SWAP ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j], af[i], acc[i][j], 0, 0, 0)
                                 : __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        // interleave the next slice's fragment reads with this slice's MFMAs
        constexpr int NR = FI + FJ, NM = FI * FJ, PER = NM / NR;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);   // PER MFMAs
        }
        __builtin_amdgcn_sched_group_barrier(0x008, NM - PER * NR, 0);
    };
    bf16x8_t a0[FI], b0[FJ], a1[FI], b1[FJ];
    land(0);
    if (S - 1 < nk) issue(S - 1);
    read(0, a0, b0);
    for (int s = 0; s < nk; s += 2) {
        step(s, a0, b0, a1, b1);
        if (s + 1 < nk) step(s + 1, a1, b1, a0, b0);
    }
    if constexpr (SWAP) {
        reg_epilogue<EPI, TM, TN, FI, FJ, WM, WN>(g, acc, m0, n0, tab);
    } else {
        // every wave's last fragment reads are done before the ring becomes the stage
        __syncthreads();
        tile_epilogue<EPI, TM, TN, FI, FJ, WM, WN>(g, acc, m0, n0, 0, sm, tab);
    }
}

// ---------------------------------------------------------------------------
// Inference through every layer in one launch (hidden width 512)
//
// A workgroup of 8 waves takes TM rows through the whole network: their
// activations stay in LDS (TM x 512 BF16, overwritten in place by each layer
// once every wave has read them), so only the input rows, the weights (from
// L2, each layer's read once per workgroup) and the outputs cross the memory
// hierarchy.  Hidden layers: wave w computes columns 64 w .. 64 w + 63 of
// all TM rows, weight fragments straight into registers three K slices
// ahead, activation fragments from LDS.  The MFMAs take the operands swapped (as in
// the inference epilogue of the layer-by-layer kernel), so a lane ends with
// 4 consecutive columns of one row: bias in the accumulators, then GELU and
// BF16 rounding written back into LDS as 8-byte groups.  The output layer:
// wave w computes 16-column block w of every row.  Same operations, operand
// order and K order as the layer-by-layer inference kernels.

constexpr int FH = 512;               // hidden width
constexpr int FUSED_MAX_OUT = 128;    // output columns (8 waves x 16)

struct FusedArgs {
    const uint16_t* X;   // [M][kin] BF16 input rows
    int M, kin, L;       // rows, padded input width (32 .. 512, multiple of 32), linear layers (2 .. MAX_LAYERS)
    int d_out;           // 1 .. FUSED_MAX_OUT
    const uint16_t* W[MAX_LAYERS];   // layer l: [npad][kpad] BF16 (kpad = kin for l = 0, else FH)
    const float* bias[MAX_LAYERS];
    float* Y;            // [M][d_out] FP32
    const f32x4_t* gelu_tab;
};

// element offset of (row r, column c) in the LDS activations: the 16-byte
// chunk index is XORed with r mod 16, so the 16 rows a fragment read
// touches at one chunk land in 16 different bank groups
__device__ __forceinline__ int fused_at(int r, int c) { return r * FH + (((c >> 3) ^ (r & 15)) << 3) + (c & 7); }

// Weight fragments of FJ row blocks (rows wrow + 16 j K, K contiguous, K / 32
// slices) go straight into registers through a ring of 4, three K slices
// ahead (loads past the last slice repeat it, unused).  fused_pre loads
// slices 0..2 (issued early, e.g. before the previous layer's epilogue);
// fused_k then runs every slice: acc[i][j] += activation row block i (from
// LDS) x weight block j.  NK > 0: the slice count, fully unrolled; NK = 0:
// K / 32 at run time, in an unconditional loop of 4 slices (so the
// compiler's waits leave three slices in flight) and a remainder.
template <int FJ>
__device__ __forceinline__ void fused_wload(const uint16_t* __restrict__ wrow, int K, int s, u32x4_t (&b)[FJ]) {
    s = min(s, (K >> 5) - 1);
#pragma unroll
    for (int j = 0; j < FJ; ++j) b[j] = *(const u32x4_t*)(wrow + (int64_t)j * 16 * K + s * 32);
}

template <int FJ>
__device__ __forceinline__ void fused_pre(const uint16_t* __restrict__ wrow, int K, u32x4_t (&w0)[FJ],
                                          u32x4_t (&w1)[FJ], u32x4_t (&w2)[FJ]) {
    fused_wload<FJ>(wrow, K, 0, w0);
    fused_wload<FJ>(wrow, K, 1, w1);
    fused_wload<FJ>(wrow, K, 2, w2);
}

template <int FI, int FJ, int NK>
__device__ __forceinline__ void fused_k(f32x4_t (&acc)[FI][FJ], const uint16_t* __restrict__ wrow, int K,
                                        const uint16_t* hs, u32x4_t (&w0)[FJ], u32x4_t (&w1)[FJ],
                                        u32x4_t (&w2)[FJ], u32x4_t (&w3)[FJ]) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, q = lane >> 4;
    auto step = [&](int s, const u32x4_t (&cur)[FJ], u32x4_t (&nxt)[FJ]) {
        fused_wload<FJ>(wrow, K, s + 3, nxt);   // into the registers slice s - 1 used
        // keep the loads here: left alone, the scheduler sinks them next to
        // their first use a ring later, which exposes their latency
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < FI; ++i) {
            const bf16x8_t af =
                __builtin_bit_cast(bf16x8_t, *(const u32x4_t*)(hs + fused_at(i * 16 + r16, s * 32 + q * 8)));
#pragma unroll
            for (int j = 0; j < FJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, cur[j]), af,
                                                                   acc[i][j], 0, 0, 0);
        }
    };
    auto four = [&](int s) {
        step(s, w0, w3);
        step(s + 1, w1, w0);
        step(s + 2, w2, w1);
        step(s + 3, w3, w2);
    };
    if constexpr (NK > 0) {
        static_assert(NK % 4 == 0, "whole rings");
#pragma unroll
        for (int s = 0; s < NK; s += 4) four(s);
    } else {
        // whole rings, then the last nk mod 4 slices (the ring ends where it
        // started, so they take the same registers)
        const int nk = K >> 5, n4 = nk & ~3;
        for (int s = 0; s < n4; s += 4) four(s);
        if (nk - n4 > 0) step(n4, w0, w3);
        if (nk - n4 > 1) step(n4 + 1, w1, w0);
        if (nk - n4 > 2) step(n4 + 2, w2, w1);
    }
}

// TM rows per workgroup (32, 64 or 128): TM / 16 row blocks of 16 per wave
template <int TM>
__global__ __launch_bounds__(512) void mlp_infer_kernel(FusedArgs a) {
    constexpr int FI = TM / 16;
    __shared__ __attribute__((aligned(1024))) uint16_t hs[TM * FH];
    __shared__ f32x4_t tab[GELU_PIECES];
    __shared__ f32x4_t bs[(MAX_LAYERS - 1) * FH / 4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int m0 = xcd_swizzle((int)blockIdx.x, (int)gridDim.x) * TM;
    const int n0 = w * 16;   // the output layer's columns of this wave
    const int lo = a.L - 1;
    // hidden weight rows 64 w + 16 j + r16, output weight rows n0 + r16
    // (present up to the padded row count), 8 K values at 32 s + 8 q
    auto hrow = [&](int l) { return a.W[l] + (int64_t)(w * 64 + r16) * (l == 0 ? a.kin : FH) + q * 8; };
    const uint16_t* orow = a.W[lo] + (int64_t)(n0 + r16) * FH + q * 8;
    u32x4_t w0[4], w1[4], w2[4], w3[4];
    fused_pre<4>(hrow(0), a.kin, w0, w1, w2);
    // input rows (rows past M repeat row M - 1; their outputs are not stored)
    const int cpr = a.kin >> 3;
    for (int e = tid; e < TM * cpr; e += 512) {
        const int r = e / cpr, c = e - r * cpr;
        const int row = min(m0 + r, a.M - 1);
        *(u32x4_t*)(hs + fused_at(r, c * 8)) = *(const u32x4_t*)(a.X + (int64_t)row * a.kin + c * 8);
    }
    static_assert(GELU_PIECES == 512, "one table piece per thread");
    tab[tid] = a.gelu_tab[tid];
    // hidden biases in LDS too (read at each layer's start without waiting
    // for weight loads in flight)
    for (int e = tid; e < (a.L - 1) * (FH / 4); e += 512) {
        const float* b = a.bias[e / (FH / 4)] + 4 * (e % (FH / 4));
        bs[e] = f32x4_t{b[0], b[1], b[2], b[3]};
    }
    __syncthreads();

    u32x4_t o0[1], o1[1], o2[1], o3[1];
    for (int l = 0; l < lo; ++l) {
        f32x4_t acc[FI][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const f32x4_t b0 = bs[l * (FH / 4) + w * 16 + j * 4 + q];
#pragma unroll
            for (int i = 0; i < FI; ++i) acc[i][j] = b0;
        }
        fused_k<FI, 4, 0>(acc, hrow(l), l == 0 ? a.kin : FH, hs, w0, w1, w2, w3);
        // the next layer's first weight slices travel during the epilogue
        if (l + 1 < lo)
            fused_pre<4>(hrow(l + 1), FH, w0, w1, w2);
        else if (n0 < a.d_out)
            fused_pre<1>(orow, FH, o0, o1, o2);
        __syncthreads();   // every wave has read this layer's inputs
#pragma unroll
        for (int i = 0; i < FI; ++i) {
            const int r = i * 16 + r16;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = w * 64 + j * 16 + 4 * q;
                const uint2 h = make_uint2(pack_bf16(gelu_tab(tab, acc[i][j][0]), gelu_tab(tab, acc[i][j][1])),
                                           pack_bf16(gelu_tab(tab, acc[i][j][2]), gelu_tab(tab, acc[i][j][3])));
                *(uint2*)(hs + fused_at(r, c)) = h;
            }
        }
        __syncthreads();
    }

    // output layer: wave w, columns n0 .. n0 + 15
    if (n0 >= a.d_out) return;
    f32x4_t acc[FI][1];
    {
        f32x4_t b0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = n0 + 4 * q + r;
            b0[r] = n < a.d_out ? a.bias[lo][n] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < FI; ++i) acc[i][0] = b0;
    }
    fused_k<FI, 1, 0>(acc, orow, FH, hs, o0, o1, o2, o3);
    const bool vec_out = (a.d_out & 3) == 0;
#pragma unroll
    for (int i = 0; i < FI; ++i) {
        const int m = m0 + i * 16 + r16, n = n0 + 4 * q;
        if (m >= a.M) continue;
        float* dst = a.Y + (int64_t)m * a.d_out + n;
        if (vec_out && n + 4 <= a.d_out) {
            *(f32x4_t*)dst = acc[i][0];
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (n + r < a.d_out) dst[r] = acc[i][0][r];
        }
    }
}

// ---------------------------------------------------------------------------
// input rows: [features | noise | zero padding] in BF16

struct InputArgs {
    const float* feats;          // [n_feats][d_feat]
    int64_t n_feats;
    const int32_t* feat_of_row;  // [logical rows] or null (feature row 0); clamped into range
    const int32_t* draw;         // [logical rows] or null (draw 0); used when draws == 0
    int draws;                   // > 0: physical row r is logical row r / draws, draw r % draws
    int d_feat, d_noise, in_pad;
    int64_t rows;
    uint32_t k0, k1;
    uint16_t* X0;                // [rows][in_pad]
    uint16_t* X0T;               // [in_pad][ldt] or null
    int64_t ldt;
};

// Two halves of the grid (blockIdx.y): the noise groups of every row, then
// the feature and zero groups, so that the waves generating noise
// (Philox and Box-Muller) do nothing else.  With draws > 0 a feature thread
// serves one logical row and writes its group to all of that row's draws
// (one feature lookup instead of one per draw).  rows * groups < 2^32 (rows
// <= 2^24, in_pad <= 512): 32-bit index arithmetic.
__device__ __forceinline__ uint2 pack4_bf16(const float (&v)[4]) {
    uint2 p;
    p.x = (uint32_t)to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16);
    p.y = (uint32_t)to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16);
    return p;
}

__device__ __forceinline__ void put_group(const InputArgs& a, uint32_t r, int c, uint2 p) {
    *(uint2*)(a.X0 + (int64_t)r * a.in_pad + c) = p;
    if (a.X0T) {
        const uint16_t h[4] = {(uint16_t)p.x, (uint16_t)(p.x >> 16), (uint16_t)p.y, (uint16_t)(p.y >> 16)};
#pragma unroll
        for (int q = 0; q < 4; ++q) a.X0T[(int64_t)(c + q) * a.ldt + r] = h[q];
    }
}

__global__ __launch_bounds__(256) void build_inputs_kernel(InputArgs a) {
    const uint32_t groups = (uint32_t)a.in_pad / 4, ng = (uint32_t)a.d_noise / 4, nf = groups - ng;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (blockIdx.y == 0) {
        if (ng == 0 || e >= (uint32_t)a.rows * ng) return;
        const uint32_t r = e / ng, gi = e - r * ng;
        const uint32_t b = a.draws > 0 ? r / (uint32_t)a.draws : r;
        const uint32_t s = a.draws > 0 ? r - b * (uint32_t)a.draws : (a.draw ? (uint32_t)a.draw[b] : 0u);
        float v[4];
        normal4(b, s, gi, a.k0, a.k1, v);
        put_group(a, r, a.d_feat + 4 * (int)gi, pack4_bf16(v));
        return;
    }
    // feature and zero groups of logical row b (physical rows b draws .. + draws - 1, or b)
    const uint32_t per_b = a.draws > 0 ? (uint32_t)a.draws : 1u;
    const uint32_t n_b = (uint32_t)a.rows / per_b;
    if (nf == 0 || e >= n_b * nf) return;
    const uint32_t b = e / nf, gi = e - b * nf;
    const int c = 4 * (int)gi < a.d_feat ? 4 * (int)gi : 4 * (int)gi + a.d_noise;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (c < a.d_feat) {
        int64_t f = a.feat_of_row ? (int64_t)a.feat_of_row[b] : 0;
        f = f < 0 ? 0 : (f >= a.n_feats ? a.n_feats - 1 : f);
        const float* src = a.feats + f * a.d_feat + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = src[q];
    }
    const uint2 p = pack4_bf16(v);
    for (uint32_t d = 0; d < per_b; ++d) put_group(a, b * per_b + d, c, p);
}

// FP32 noise rows (the generator alone): out[r][j], counter words (r, draw[r])
__global__ __launch_bounds__(256) void noise_kernel(const int32_t* draw, int64_t rows, int d_noise, uint32_t k0,
                                                    uint32_t k1, float* out) {
    const int groups = d_noise / 4;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * groups) return;
    const int64_t r = e / groups;
    const int gi = (int)(e % groups);
    float z[4];
    normal4((uint32_t)r, draw ? (uint32_t)draw[r] : 0u, (uint32_t)gi, k0, k1, z);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[r * d_noise + gi * 4 + q] = z[q];
}

// ---------------------------------------------------------------------------
// IMLE: nearest of S draws per target by the (optionally weighted) squared
// distance (one wave per target; lowest index on ties)

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Upstream gradient of the output layer in BF16, both orientations, for
// row b, by one wave.  With targets: g = scale w (y - t) and the row's sum
// of w (y - t)^2 (w = 1 when wt is null); without: g = y.
__device__ __forceinline__ void out_grad_row(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ wt, int d_out, int out_pad, float scale,
                                             uint16_t* __restrict__ GY, uint16_t* __restrict__ GYT, int64_t ldt,
                                             int64_t b, float* __restrict__ row_loss) {
    const int lane = threadIdx.x & 63;
    float acc = 0.f;
    for (int d = lane; d < out_pad; d += 64) {
        float gv = 0.f;
        if (d < d_out) {
            if (t) {
                const float w = wt ? wt[d] : 1.f;
                const float df = y[d] - t[d];
                acc += w * df * df;
                gv = scale * (w * df);
            } else {
                gv = y[d];
            }
        }
        const uint16_t h = to_bf16(gv);
        GY[b * out_pad + d] = h;
        GYT[(int64_t)d * ldt + b] = h;
    }
    if (t && row_loss) {
        acc = wave_sum(acc);
        if (lane == 0) row_loss[b] = acc;
    }
}

// the same for every row of Y (a wave per row)
__global__ __launch_bounds__(256) void out_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                       const float* __restrict__ W, int d_out, int out_pad,
                                                       int64_t rows, float scale,
                                                       uint16_t* __restrict__ GY, uint16_t* __restrict__ GYT,
                                                       int64_t ldt, float* __restrict__ row_loss) {
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= rows) return;
    out_grad_row(Y + b * d_out, T ? T + b * d_out : nullptr, W ? W + b * d_out : nullptr, d_out, out_pad, scale,
                 GY, GYT, ldt, b, row_loss);
}

// Nearest draw per target (IMLE): chosen[b] = argmin over the S draws s of
// sum_d w_d (Y[b S + s][d] - T[b][d])^2 (w = 1 when W is null; lowest s
// among equals).  One workgroup per target: with S <= 256 the draws are
// spread over the 256 lanes (P = 256 / S lanes per draw, each summing every
// P-th dimension), so four waves' loads are in flight together and each
// lane's chain is d_out / P long; the P partial sums of a draw are added in
// lane order through LDS and the first wave finds the minimum.  More than
// 256 draws: the first wave takes one draw after another.  Then, for the
// chosen draw, what the rest of a training step needs of it: the first
// wave writes the squared-error gradient of its output (out_grad_row, from
// the output already in Y), the second its input row for the second pass
// (the values build_inputs_kernel would write for logical row b, draw
// chosen[b]).
struct SelectArgs {
    const float* Y;       // [B S][d_out]
    const float* T;       // [B][d_out]
    const float* W;       // [B][d_out] or null
    int d_out;
    int64_t B;
    int S;
    int32_t* chosen;      // [B]
    int out_pad;          // gradient rows [B][out_pad] and columns [out_pad][ldt]
    float scale;
    uint16_t *GY, *GYT;
    int64_t ldt;
    float* row_loss;      // [B]
    InputArgs in;         // X0, X0T (ldt) for rows b = 0..B-1
};

// the kept row's input row for draw s (what build_inputs_kernel writes for
// logical row b, draw s), one wave
__device__ __forceinline__ void select_input_row(const InputArgs& in, int64_t b, int s) {
    const int lane = threadIdx.x & 63;
    for (int gi = lane; gi < in.in_pad / 4; gi += 64) {
        const int c = 4 * gi;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (c >= in.d_feat && c < in.d_feat + in.d_noise) {
            normal4((uint32_t)b, (uint32_t)s, (uint32_t)(c - in.d_feat) / 4u, in.k0, in.k1, v);
        } else if (c < in.d_feat) {
            int64_t f = in.feat_of_row ? (int64_t)in.feat_of_row[b] : 0;
            f = f < 0 ? 0 : (f >= in.n_feats ? in.n_feats - 1 : f);
            const float* src = in.feats + f * in.d_feat + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = src[q];
        }
        put_group(in, (uint32_t)b, c, pack4_bf16(v));
    }
}

__global__ __launch_bounds__(256) void imle_select_kernel(SelectArgs a) {
    __shared__ float part[256];
    __shared__ int pick;
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    if (b >= a.B) return;   // workgroup-uniform
    const int d_out = a.d_out, S = a.S;
    const float* t = a.T + b * d_out;
    const float* wt = a.W ? a.W + b * d_out : nullptr;
    if (S <= 256) {
        const int P = 256 / S;
        const int s = tid / P, q = tid - s * P;
        float acc = 0.f;
        if (s < S) {
            const float* y = a.Y + (b * S + s) * d_out;
            for (int d = q; d < d_out; d += P) {
                const float df = y[d] - t[d];
                acc += (wt ? wt[d] : 1.f) * df * df;
            }
        }
        part[tid] = acc;
        __syncthreads();
        if (tid < 64) {
            float dist = INFINITY;
            int idx = 256;
            for (int i = lane; i < S; i += 64) {   // increasing draws: strict < keeps the lowest among equals
                float sum = 0.f;
                for (int j = 0; j < P; ++j) sum += part[i * P + j];
                if (sum < dist) {
                    dist = sum;
                    idx = i;
                }
            }
            // argmin across the wave, lowest draw among equal distances
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const float od = __shfl_xor(dist, o);
                const int oi = __shfl_xor(idx, o);
                if (od < dist || (od == dist && oi < idx)) {
                    dist = od;
                    idx = oi;
                }
            }
            if (lane == 0) pick = idx;
        }
    } else if (tid < 64) {
        float best = 0.f;
        int bi = 0;
        for (int s = 0; s < S; ++s) {
            const float* y = a.Y + (b * S + s) * d_out;
            float acc = 0.f;
            for (int d = lane; d < d_out; d += 64) {
                const float df = y[d] - t[d];
                acc += (wt ? wt[d] : 1.f) * df * df;
            }
            acc = wave_sum(acc);
            if (s == 0 || acc < best) {
                best = acc;
                bi = s;
            }
        }
        if (lane == 0) pick = bi;
    }
    __syncthreads();
    // the chosen draw: its loss gradient (first wave), its input row (second)
    const int s = pick;
    if (tid < 64) {
        if (lane == 0) a.chosen[b] = s;
        out_grad_row(a.Y + (b * S + s) * d_out, t, wt, d_out, a.out_pad, a.scale, a.GY, a.GYT, a.ldt, b,
                     a.row_loss);
    } else if (tid < 128) {
        select_input_row(a.in, b, s);
    }
}

// The end of a backward pass, every layer in one launch: blockIdx.y = 0
// sums each split-K layer's weight-gradient partials in split order,
// blockIdx.y = 1 forms each layer's bias gradient as the row sum of its
// BF16 output gradient D^T (one wave per output, rows % 8 == 0 and
// ldt % 8 == 0 read as 16-byte chunks), and block (0, 2), when a loss is
// asked for, reduces the per-row losses (loss_reduce).
struct GradFinishArgs {
    int L;
    int64_t rows, ldt;
    int64_t estart[MAX_LAYERS + 1];   // prefix sums of the split-K layers' M N (0 for the others), each
                                      // rounded up to a multiple of 256
    int64_t ostart[MAX_LAYERS + 1];   // prefix sums of dout, each rounded up to a multiple of 4
    int64_t ecount[MAX_LAYERS];       // M N of a split-K layer
    int dout[MAX_LAYERS];
    int ksplit[MAX_LAYERS];
    const float* part[MAX_LAYERS];    // [ksplit][M N] partials of a split-K layer
    float* dW[MAX_LAYERS];
    const uint16_t* DT[MAX_LAYERS];   // [dout][ldt]
    float* gb[MAX_LAYERS];
    const float* row_loss;            // null: no loss
    float loss_scale;
    float* loss;
};

// loss = inv * sum of the row sums (one workgroup, fixed summation order)
__device__ __forceinline__ void loss_reduce(const float* __restrict__ row_loss, int64_t rows, float inv,
                                            float* __restrict__ loss) {
    __shared__ float red[256];
    float acc = 0.f;
    for (int64_t r = threadIdx.x; r < rows; r += 256) acc += row_loss[r];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * inv;
}

// Each layer's ranges start at multiples of 256 (partials) and 4 (bias
// outputs, one wave each), so a workgroup lies in one layer and the layer
// search runs on the workgroup index (scalar loads of the arguments).
__global__ __launch_bounds__(256) void grad_finish_kernel(GradFinishArgs a) {
    if (blockIdx.y == 2) {
        if (blockIdx.x == 0 && a.row_loss) loss_reduce(a.row_loss, a.rows, a.loss_scale, a.loss);
        return;
    }
    if (blockIdx.y == 0) {
        const int64_t e0 = (int64_t)blockIdx.x * 256;
        if (e0 >= a.estart[a.L]) return;
        int l = 0;
        while (e0 >= a.estart[l + 1]) ++l;
        const int64_t cnt = a.ecount[l], i = e0 + threadIdx.x - a.estart[l];
        if (i >= cnt) return;
        float acc = 0.f;
        for (int s = 0; s < a.ksplit[l]; ++s) acc += a.part[l][(int64_t)s * cnt + i];
        a.dW[l][i] = acc;
        return;
    }
    const int64_t ob0 = (int64_t)blockIdx.x * 4;
    const int lane = threadIdx.x & 63;
    if (ob0 >= a.ostart[a.L]) return;
    int l = 0;
    while (ob0 >= a.ostart[l + 1]) ++l;
    const int64_t o = ob0 + (threadIdx.x >> 6) - a.ostart[l];
    if (o >= a.dout[l]) return;
    const uint16_t* src = a.DT[l] + o * a.ldt;
    float acc = 0.f;
    if (a.rows % 8 == 0 && a.ldt % 8 == 0) {
        // 16-byte chunks: every lane's loads are independent and in flight together
        for (int64_t c = lane; c < a.rows / 8; c += 64) {
            const u32x4_t v = *(const u32x4_t*)(src + 8 * c);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc += __uint_as_float(v[q] << 16) + __uint_as_float(v[q] & 0xFFFF0000u);
        }
    } else {
        for (int64_t r = lane; r < a.rows; r += 64) acc += __uint_as_float((uint32_t)src[r] << 16);
    }
    acc = wave_sum(acc);
    if (lane == 0) a.gb[l][o] = acc;
}

// Adam over every parameter and the BF16 weight copies of the updated
// weights in one launch: elements [0, wend) walk each layer's padded
// [npad][kpad] block (Adam on the real [dout][din] part, then Wb and WbT;
// zeros in the padding), elements [wend, wend + bias count) the biases.
// Adam with bias correction (bc1, bc2 = 1 - beta^t), then the BF16 copy.
struct AdamRefreshArgs {
    float *P, *Mo, *Vo;
    const float* G;
    float lr, b1, b2, eps, gscale, bc1, bc2;
    int L;
    int64_t wstart[MAX_LAYERS + 1];   // prefix sums of npad * kpad, each rounded up to a multiple of 256
    int64_t bstart[MAX_LAYERS + 1];   // prefix sums of dout, each rounded up to a multiple of 256
    int din[MAX_LAYERS], dout[MAX_LAYERS], kpad[MAX_LAYERS], npad[MAX_LAYERS];
    int64_t woff[MAX_LAYERS], boff[MAX_LAYERS];
    uint16_t* Wb[MAX_LAYERS];
    uint16_t* WbT[MAX_LAYERS];   // null: none kept for that layer
};

__device__ __forceinline__ float adam_one(const AdamRefreshArgs& a, int64_t idx) {
    const float g = a.gscale * a.G[idx];
    const float m = a.b1 * a.Mo[idx] + (1.f - a.b1) * g;
    const float v = a.b2 * a.Vo[idx] + (1.f - a.b2) * g * g;
    a.Mo[idx] = m;
    a.Vo[idx] = v;
    const float p = a.P[idx] - a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
    a.P[idx] = p;
    return p;
}

// Every layer's range starts at a multiple of 256, so a workgroup lies in
// one layer: the layer search runs on the workgroup index (scalar loads of
// the arguments), not per lane.
__global__ __launch_bounds__(256) void adam_refresh_kernel(AdamRefreshArgs a) {
    const int64_t e0 = (int64_t)blockIdx.x * 256, e = e0 + threadIdx.x;
    if (e0 < a.wstart[a.L]) {
        int l = 0;
        while (e0 >= a.wstart[l + 1]) ++l;
        const int64_t loc = e - a.wstart[l];
        if (loc >= (int64_t)a.npad[l] * a.kpad[l]) return;
        const int o = (int)loc / a.kpad[l], i = (int)loc - o * a.kpad[l];
        uint16_t v = 0;
        if (o < a.dout[l] && i < a.din[l]) v = to_bf16(adam_one(a, a.woff[l] + (int64_t)o * a.din[l] + i));
        a.Wb[l][loc] = v;
        if (a.WbT[l]) a.WbT[l][(int64_t)i * a.npad[l] + o] = v;
        return;
    }
    const int64_t b0 = e0 - a.wstart[a.L];
    if (b0 >= a.bstart[a.L]) return;
    int l = 0;
    while (b0 >= a.bstart[l + 1]) ++l;
    const int64_t j = e - a.wstart[a.L] - a.bstart[l];
    if (j < a.dout[l]) adam_one(a, a.boff[l] + j);
}

// BF16 copies of one layer's weights: Wb [npad][kpad] and WbT [kpad][npad]
// (null to skip), zero outside the real [dout][din] block
__global__ __launch_bounds__(256) void refresh_kernel(const float* __restrict__ W, int din, int dout, int kpad,
                                                      int npad, uint16_t* __restrict__ Wb, uint16_t* __restrict__ WbT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)npad * kpad) return;
    const int o = (int)(e / kpad), i = (int)(e % kpad);
    const uint16_t v = (o < dout && i < din) ? to_bf16(W[(int64_t)o * din + i]) : (uint16_t)0;
    Wb[e] = v;
    if (WbT) WbT[(int64_t)i * npad + o] = v;
}

// seeds: x = y std + mean, angles wrapped into [-pi, pi), clamped into
// [lo, hi].  A workgroup takes 64 particles and walks their outputs 64 at a
// time through an LDS tile: rows of Y read coalesced along the outputs,
// the dimension-major X (and zeroed M, V) written coalesced along the
// particles.
constexpr int SEED_TILE = 64;

__global__ __launch_bounds__(256) void sample_store_kernel(const float* __restrict__ Y, int d_out, int64_t n,
                                                           const float* __restrict__ mean,
                                                           const float* __restrict__ stdv,
                                                           const float* __restrict__ lo, const float* __restrict__ hi,
                                                           const uint8_t* __restrict__ wrap, float* __restrict__ X,
                                                           float* __restrict__ M, float* __restrict__ V, int64_t ld) {
    __shared__ float tile[SEED_TILE][SEED_TILE + 1];
    const int64_t i0 = (int64_t)blockIdx.x * SEED_TILE;
    const int t = threadIdx.x;
    for (int d0 = 0; d0 < d_out; d0 += SEED_TILE) {
        for (int e = t; e < SEED_TILE * SEED_TILE; e += 256) {
            const int p = e / SEED_TILE, q = e % SEED_TILE;
            const int64_t i = i0 + p;
            tile[p][q] = (i < n && d0 + q < d_out) ? Y[i * d_out + d0 + q] : 0.f;
        }
        __syncthreads();
        for (int e = t; e < SEED_TILE * SEED_TILE; e += 256) {
            const int q = e / SEED_TILE, p = e % SEED_TILE, d = d0 + q;
            const int64_t i = i0 + p;
            if (i < n && d < d_out) {
                float x = tile[p][q] * stdv[d] + mean[d];
                if (wrap && wrap[d]) x -= 6.283185307179586f * floorf((x + 3.14159265358979f) * 0.15915494309189535f);
                x = fminf(fmaxf(x, lo[d]), hi[d]);
                X[d * ld + i] = x;
                if (M) M[d * ld + i] = 0.f;
                if (V) V[d * ld + i] = 0.f;
            }
        }
        __syncthreads();
    }
}

}  // namespace mlp
}  // namespace ct
