// C ABI of the learned seed proposer (declared in cutamp.h): handle, weights,
// forward / backward / Adam, one IMLE training step, and seeding particles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "cutamp.h"
#include "mlp_kernels.hpp"

namespace {

using namespace ct::mlp;

constexpr int64_t PART_CAP = int64_t(16) << 20;   // split-K partial floats (64 MiB)

int64_t up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
int err_of(hipError_t e) { return e == hipSuccess ? CT_OK : CT_ERR_DEVICE; }
unsigned blocks(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

struct ct_mlp {
    ct_mlp_shape s{};
    int L = 0;                // linear layers = depth + 1
    int d_in = 0, in_pad = 0, out_pad = 0;
    int64_t rows_cap = 0;     // max_rows rounded up to 64
    std::vector<int> din, dout, kpad, npad;
    std::vector<int64_t> woff, boff;
    int64_t n_params = 0;
    float *P = nullptr, *Mo = nullptr, *Vo = nullptr, *G = nullptr;
    std::vector<uint16_t*> Wb, WbT;
    uint16_t *X0 = nullptr, *X0T = nullptr;
    std::vector<float*> Z;
    std::vector<uint16_t*> H, HT, D, DT;
    float* Y = nullptr;
    uint16_t *GY = nullptr, *GYT = nullptr;
    float* part = nullptr;
    int64_t part_cap = 0;   // floats in part
    f32x4_t* gelu_tab = nullptr;   // GELU_PIECES cubic pieces of the normal CDF
    float* row_loss = nullptr;
    int32_t* chosen = nullptr;
    int64_t fwd_rows = -1;    // rows of the last forward that kept its activations
    std::vector<void*> allocs;

    template <class T>
    bool alloc(T*& p, int64_t count) {
        void* q = nullptr;
        if (hipMalloc(&q, (size_t)count * sizeof(T)) != hipSuccess) return false;
        if (hipMemset(q, 0, (size_t)count * sizeof(T)) != hipSuccess) {
            (void)hipFree(q);
            return false;
        }
        allocs.push_back(q);
        p = (T*)q;
        return true;
    }
    ~ct_mlp() {
        for (void* q : allocs) (void)hipFree(q);
    }
};

namespace {

bool shape_ok(const ct_mlp_shape& s) {
    return s.d_feat >= 0 && s.d_feat % 4 == 0 && s.d_noise >= 0 && s.d_noise % 4 == 0 && s.d_feat + s.d_noise > 0 &&
           s.d_feat + s.d_noise <= 512 &&
           s.hidden >= 64 && s.hidden % 64 == 0 && s.hidden <= 4096 && s.depth >= 1 && s.depth <= 8 &&
           s.d_out >= 1 && s.d_out <= 512 && s.max_rows >= 64 && s.max_rows % 64 == 0 &&
           s.max_rows <= (int64_t(1) << 24);
}

// rows from which the 256 x 256 tiles keep at least half the compute units
// busy at N = 512 (128 workgroups); below, the 32 x 32 tiles
constexpr int BIG_ROWS = 16384;

template <int TILE, int BK>
int gemm_tile(const GemmArgs& g, hipStream_t st) {
    const unsigned grid = (unsigned)(((g.M + TILE - 1) / TILE) * ((g.N + TILE - 1) / TILE) * g.ksplit);
    hipLaunchKernelGGL((gemm_nt_kernel<EPI_DW, TILE, BK>), dim3(grid), dim3(256), 0, st, g);
    return err_of(hipGetLastError());
}

template <int TM, int TN, int WM, int WN, int S>
int gemm_pipe(int epi, const GemmArgs& g, hipStream_t st) {
    const unsigned grid = (unsigned)(((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN));
    const dim3 block(64 * WM * WN);
    switch (epi) {
        case EPI_HID_TRAIN:
            hipLaunchKernelGGL((gemm_pipe_kernel<EPI_HID_TRAIN, TM, TN, WM, WN, S>), dim3(grid), block, 0, st, g); break;
        case EPI_HID_INFER:
            hipLaunchKernelGGL((gemm_pipe_kernel<EPI_HID_INFER, TM, TN, WM, WN, S>), dim3(grid), block, 0, st, g); break;
        case EPI_BWD:
            hipLaunchKernelGGL((gemm_pipe_kernel<EPI_BWD, TM, TN, WM, WN, S>), dim3(grid), block, 0, st, g); break;
        default: hipLaunchKernelGGL((gemm_pipe_kernel<EPI_OUT, TM, TN, WM, WN, S>), dim3(grid), block, 0, st, g); break;
    }
    return err_of(hipGetLastError());
}

// Forward and backward products run the direct-to-LDS pipelined kernel:
// 256 x 256 tiles (8 waves) for hidden layers over many rows, 128 x 128 for
// the output layer there, and below (the fitted passes of a training step)
// 32 x 32 tiles of four 16 x 16 waves with a 3-slice ring: these passes are
// bound by load latency, and 512 workgroups of 4 waves at 1,024 x 512 keep
// more loads in flight than 32 x 64 tiles of two waves (a training step
// 155 us instead of 180).  Weight gradients take split-K over the
// double-buffered kernel: 32 x 32 tiles with K slices 64 deep (a training
// step 152 us instead of 155 with 64 x 64 tiles), 64 x 64 tiles with
// slices 32 deep where a K chunk is not a multiple of 64.
int gemm(int epi, const GemmArgs& g, hipStream_t st) {
    if (epi == EPI_DW) {
        const bool deep = (g.K / g.ksplit) % 64 == 0;
        return deep ? gemm_tile<GT, 64>(g, st) : gemm_tile<GT_SHALLOW, 32>(g, st);
    }
    if (g.ksplit != 1) return CT_ERR_INVALID_ARG;
    if (g.M >= BIG_ROWS && epi != EPI_BWD) {
        if (g.N > 128) return gemm_pipe<256, 256, 4, 2, 4>(epi, g, st);
        return gemm_pipe<128, 128, 2, 2, 4>(epi, g, st);
    }
    return gemm_pipe<32, 32, 2, 2, 3>(epi, g, st);
}

// split-K factor of a weight-gradient product: enough workgroups to cover
// the chip (about 512), each K chunk a multiple of 32, at most 8 chunks (the
// partials are read back once more), partials within the space left
int pick_ksplit(int M, int N, int64_t K, int64_t cap) {
    const int64_t tiles = (int64_t)((M + GT - 1) / GT) * ((N + GT - 1) / GT);
    int s = 1;
    while (tiles * s < 512 && K % (int64_t(GK) * s * 2) == 0 && (int64_t)s * 2 * M * N <= cap && s < 8) s *= 2;
    return s;
}

int refresh(ct_mlp* m, hipStream_t st) {
    for (int l = 0; l < m->L; ++l) {
        const int64_t cnt = (int64_t)m->npad[l] * m->kpad[l];
        hipLaunchKernelGGL(refresh_kernel, dim3(blocks(cnt, 256)), dim3(256), 0, st, m->P + m->woff[l], m->din[l],
                           m->dout[l], m->kpad[l], m->npad[l], m->Wb[l], m->WbT[l]);
    }
    return err_of(hipGetLastError());
}

// every layer in one launch (activations kept in LDS): hidden width 512, at
// most FUSED_MAX_OUT outputs, 8,192 rows or more.  Each workgroup reads
// every weight once from L2, so blocks are as tall as 256 workgroups allow
// (128 rows from 32,768 rows, 64 from 16,384, else 32); below 8,192 rows the
// per-layer launches are faster.
bool fused_ok(const ct_mlp* m, int64_t rows) {
    return m->s.hidden == FH && m->s.d_out <= FUSED_MAX_OUT && rows >= 256 * 32;
}

int infer_fused(ct_mlp* m, int64_t rows, hipStream_t st) {
    FusedArgs f{};
    f.X = m->X0;
    f.M = (int)rows;
    f.kin = m->in_pad;
    f.L = m->L;
    f.d_out = m->s.d_out;
    for (int l = 0; l < m->L; ++l) {
        f.W[l] = m->Wb[l];
        f.bias[l] = m->P + m->boff[l];
    }
    f.Y = m->Y;
    f.gelu_tab = m->gelu_tab;
    if (rows >= 256 * 128)
        hipLaunchKernelGGL(mlp_infer_kernel<128>, dim3(blocks(rows, 128)), dim3(512), 0, st, f);
    else if (rows >= 256 * 64)
        hipLaunchKernelGGL(mlp_infer_kernel<64>, dim3(blocks(rows, 64)), dim3(512), 0, st, f);
    else
        hipLaunchKernelGGL(mlp_infer_kernel<32>, dim3(blocks(rows, 32)), dim3(512), 0, st, f);
    return err_of(hipGetLastError());
}

// where the input rows go (X0, and X0^T when training) and what they hold
InputArgs input_args(const ct_mlp* m, const float* feats, int64_t n_feats, const int32_t* feat_of_row,
                     const int32_t* draw, int draws, int64_t rows, uint64_t seed, bool train) {
    InputArgs a{};
    a.feats = feats;
    a.n_feats = n_feats;
    a.feat_of_row = feat_of_row;
    a.draw = draw;
    a.draws = draws;
    a.d_feat = m->s.d_feat;
    a.d_noise = m->s.d_noise;
    a.in_pad = m->in_pad;
    a.rows = rows;
    a.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(seed >> 32);
    a.X0 = m->X0;
    a.X0T = train ? m->X0T : nullptr;
    a.ldt = m->rows_cap;
    return a;
}

// inputs + every layer (out_layer false: the hidden layers only; build
// false: the input rows are already in X0 / X0^T); train keeps Z, H, H^T
// and X0^T for the backward pass
int forward(ct_mlp* m, const float* feats, int64_t n_feats, const int32_t* feat_of_row, const int32_t* draw,
            int draws, int64_t rows, uint64_t seed, bool train, hipStream_t st, bool out_layer = true,
            bool build = true) {
    int rc = CT_OK;
    if (build) {
        const InputArgs a = input_args(m, feats, n_feats, feat_of_row, draw, draws, rows, seed, train);
        const int ng = m->s.d_noise / 4, nf = m->in_pad / 4 - ng;
        hipLaunchKernelGGL(build_inputs_kernel, dim3(blocks(rows * std::max(ng, nf), 256), 2), dim3(256), 0, st, a);
        rc = err_of(hipGetLastError());
    }
    if (!train && fused_ok(m, rows)) {
        m->fwd_rows = -1;
        return rc == CT_OK ? infer_fused(m, rows, st) : rc;
    }
    for (int l = 0; l < (out_layer ? m->L : m->L - 1) && rc == CT_OK; ++l) {
        GemmArgs g{};
        g.A = l == 0 ? m->X0 : m->H[l - 1];
        g.lda = l == 0 ? m->in_pad : m->s.hidden;
        g.B = m->Wb[l];
        g.ldb = m->kpad[l];
        g.M = (int)rows;
        g.N = m->dout[l];
        g.K = m->kpad[l];
        g.ksplit = 1;
        g.bias = m->P + m->boff[l];
        g.gelu_tab = m->gelu_tab;
        if (l + 1 < m->L) {
            g.F = m->Z[l];
            g.ldf = m->s.hidden;
            g.Hb = m->H[l];
            g.ldh = m->s.hidden;
            g.Ht = m->HT[l];
            g.ldht = m->rows_cap;
            rc = gemm(train ? EPI_HID_TRAIN : EPI_HID_INFER, g, st);
        } else {
            g.F = m->Y;
            g.ldf = m->s.d_out;
            rc = gemm(EPI_OUT, g, st);
        }
    }
    m->fwd_rows = (rc == CT_OK && train) ? rows : -1;
    return rc;
}

// gradient of sum(G * Y) from the BF16 upstream gradient already in GY / GYT
// (with loss: the loss of the rows' row_loss, scaled by inv, in the same launch
// that finishes the gradients)
int backward(ct_mlp* m, int64_t rows, hipStream_t st, float* loss = nullptr, float inv = 0.f) {
    int rc = CT_OK;
    GradFinishArgs fin{};
    fin.L = m->L;
    fin.rows = rows;
    fin.ldt = m->rows_cap;
    fin.row_loss = loss ? m->row_loss : nullptr;
    fin.loss_scale = inv;
    fin.loss = loss;
    int64_t used = 0;   // partial floats handed out so far (every layer's stay until the finish)
    DwLayers dws{};     // the weight-gradient products, run together after the backward products
    for (int l = m->L - 1; l >= 0 && rc == CT_OK; --l) {
        const bool top = l == m->L - 1;
        const uint16_t* Dm = top ? m->GY : m->D[l];     // [rows][npad]
        const uint16_t* Dt = top ? m->GYT : m->DT[l];   // [npad][rows_cap]
        // dW_l = D^T * H_{l-1} (launched after the loop): split-K partials,
        // summed with the bias gradients at the end
        GemmArgs g{};
        g.A = Dt;
        g.lda = m->rows_cap;
        g.B = l == 0 ? m->X0T : m->HT[l - 1];
        g.ldb = m->rows_cap;
        g.M = m->dout[l];
        g.N = m->din[l];
        g.K = (int)rows;
        g.ksplit = pick_ksplit(g.M, g.N, rows, m->part_cap - used);
        float* dW = m->G + m->woff[l];
        fin.ksplit[l] = g.ksplit;
        fin.dW[l] = dW;
        fin.DT[l] = Dt;
        fin.gb[l] = m->G + m->boff[l];
        if (g.ksplit == 1) {
            g.F = dW;
            g.ldf = m->din[l];
            g.fsplit = 0;
        } else {
            g.F = m->part + used;
            g.ldf = m->din[l];
            g.fsplit = (int64_t)g.M * g.N;
            fin.part[l] = g.F;
            used += g.ksplit * g.fsplit;
        }
        dws.g[l] = g;
        if (l == 0) break;
        // D_{l-1} = (D_l * W_l) . gelu'(Z_{l-1})
        GemmArgs b{};
        b.A = Dm;
        b.lda = m->npad[l];
        b.B = m->WbT[l];
        b.ldb = m->npad[l];
        b.M = (int)rows;
        b.N = m->din[l];
        b.K = m->npad[l];
        b.ksplit = 1;
        b.Zin = m->Z[l - 1];
        b.ldzin = m->s.hidden;
        b.Hb = m->D[l - 1];
        b.ldh = m->s.hidden;
        b.Ht = m->DT[l - 1];
        b.ldht = m->rows_cap;
        rc = gemm(EPI_BWD, b, st);
    }
    if (rc != CT_OK) return rc;
    // dW_l = D_l^T H_{l-1} of every layer in one launch when every K chunk is
    // 64 deep, else one launch per layer
    bool deep = true;
    dws.L = m->L;
    for (int l = 0; l < m->L; ++l) {
        const GemmArgs& g = dws.g[l];
        deep = deep && (g.K / g.ksplit) % 64 == 0;
        dws.bstart[l + 1] = dws.bstart[l] + ((g.M + GT - 1) / GT) * ((g.N + GT - 1) / GT) * g.ksplit;
    }
    if (deep) {
        hipLaunchKernelGGL(gemm_dw_layers_kernel<64>, dim3((unsigned)dws.bstart[m->L]), dim3(256), 0, st, dws);
        rc = err_of(hipGetLastError());
    } else {
        for (int l = 0; l < m->L && rc == CT_OK; ++l) rc = gemm(EPI_DW, dws.g[l], st);
    }
    if (rc != CT_OK) return rc;
    for (int l = 0; l < m->L; ++l) {
        fin.ecount[l] = fin.ksplit[l] > 1 ? (int64_t)m->dout[l] * m->din[l] : 0;
        fin.dout[l] = m->dout[l];
        fin.estart[l + 1] = fin.estart[l] + up(fin.ecount[l], 256);
        fin.ostart[l + 1] = fin.ostart[l] + up(m->dout[l], 4);
    }
    const int64_t nb = std::max(blocks(fin.estart[m->L], 256), blocks(fin.ostart[m->L], 4));
    hipLaunchKernelGGL(grad_finish_kernel, dim3((unsigned)nb, loss ? 3 : 2), dim3(256), 0, st, fin);
    return err_of(hipGetLastError());
}

int adam(ct_mlp* m, int64_t t, const ct_adam* ad, hipStream_t st) {
    const double bc1 = 1.0 - std::pow((double)ad->beta1, (double)t);
    const double bc2 = 1.0 - std::pow((double)ad->beta2, (double)t);
    AdamRefreshArgs a{};
    a.P = m->P;
    a.Mo = m->Mo;
    a.Vo = m->Vo;
    a.G = m->G;
    a.lr = ad->lr;
    a.b1 = ad->beta1;
    a.b2 = ad->beta2;
    a.eps = ad->eps;
    a.gscale = ad->grad_scale;
    a.bc1 = (float)bc1;
    a.bc2 = (float)bc2;
    a.L = m->L;
    for (int l = 0; l < m->L; ++l) {
        a.wstart[l + 1] = a.wstart[l] + up((int64_t)m->npad[l] * m->kpad[l], 256);
        a.bstart[l + 1] = a.bstart[l] + up(m->dout[l], 256);
        a.din[l] = m->din[l];
        a.dout[l] = m->dout[l];
        a.kpad[l] = m->kpad[l];
        a.npad[l] = m->npad[l];
        a.woff[l] = m->woff[l];
        a.boff[l] = m->boff[l];
        a.Wb[l] = m->Wb[l];
        a.WbT[l] = m->WbT[l];
    }
    const int64_t total = a.wstart[m->L] + a.bstart[m->L];
    hipLaunchKernelGGL(adam_refresh_kernel, dim3(blocks(total, 256)), dim3(256), 0, st, a);
    return err_of(hipGetLastError());
}

bool adam_ok(const ct_adam* a) {
    return a && std::isfinite(a->lr) && a->lr >= 0 && a->beta1 >= 0 && a->beta1 < 1 && a->beta2 >= 0 &&
           a->beta2 < 1 && a->eps > 0 && std::isfinite(a->grad_scale);
}

}  // namespace

extern "C" {

int ct_mlp_create(const ct_mlp_shape* shape, ct_mlp** out) {
    if (!shape || !out) return CT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!shape_ok(*shape)) return CT_ERR_INVALID_ARG;
    ct_mlp* m = new (std::nothrow) ct_mlp;
    if (!m) return CT_ERR_ALLOC;
    m->s = *shape;
    m->L = shape->depth + 1;
    m->d_in = shape->d_feat + shape->d_noise;
    m->in_pad = (int)up(m->d_in, GK);
    m->out_pad = (int)up(shape->d_out, GK);
    m->rows_cap = up(shape->max_rows, 64);
    for (int l = 0; l < m->L; ++l) {
        const int di = l == 0 ? m->d_in : shape->hidden;
        const int dn = l + 1 < m->L ? shape->hidden : shape->d_out;
        m->din.push_back(di);
        m->dout.push_back(dn);
        m->kpad.push_back(l == 0 ? m->in_pad : shape->hidden);
        m->npad.push_back(l + 1 < m->L ? shape->hidden : m->out_pad);
        m->woff.push_back(m->n_params);
        m->n_params += (int64_t)di * dn;
        m->boff.push_back(m->n_params);
        m->n_params += dn;
    }
    const int64_t R = m->rows_cap, Hd = shape->hidden;
    bool ok = m->alloc(m->P, m->n_params) && m->alloc(m->Mo, m->n_params) && m->alloc(m->Vo, m->n_params) &&
              m->alloc(m->G, m->n_params) && m->alloc(m->X0, R * m->in_pad) && m->alloc(m->X0T, R * m->in_pad) &&
              m->alloc(m->Y, R * shape->d_out) && m->alloc(m->GY, R * m->out_pad) &&
              m->alloc(m->GYT, R * m->out_pad) && m->alloc(m->row_loss, R) && m->alloc(m->chosen, R);
    int64_t part = 0;
    for (int l = 0; l < m->L; ++l) part = std::max(part, (int64_t)m->din[l] * m->dout[l]);
    m->part_cap = std::min<int64_t>(PART_CAP, 64 * part);
    ok = ok && m->alloc(m->part, m->part_cap);
    m->Wb.assign(m->L, nullptr);
    m->WbT.assign(m->L, nullptr);
    for (int l = 0; l < m->L && ok; ++l) {
        ok = m->alloc(m->Wb[l], (int64_t)m->npad[l] * m->kpad[l]);
        if (ok && l > 0) ok = m->alloc(m->WbT[l], (int64_t)m->npad[l] * m->kpad[l]);
    }
    m->Z.assign(shape->depth, nullptr);
    m->H.assign(shape->depth, nullptr);
    m->HT.assign(shape->depth, nullptr);
    m->D.assign(shape->depth, nullptr);
    m->DT.assign(shape->depth, nullptr);
    for (int l = 0; l < shape->depth && ok; ++l)
        ok = m->alloc(m->Z[l], R * Hd) && m->alloc(m->H[l], R * Hd) && m->alloc(m->HT[l], R * Hd) &&
             m->alloc(m->D[l], R * Hd) && m->alloc(m->DT[l], R * Hd);
    ok = ok && m->alloc(m->gelu_tab, GELU_PIECES);
    if (!ok) {
        delete m;
        return CT_ERR_ALLOC;
    }
    hipLaunchKernelGGL(gelu_table_kernel, dim3(blocks(GELU_PIECES, 256)), dim3(256), 0, 0, m->gelu_tab);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        delete m;
        return CT_ERR_DEVICE;
    }
    *out = m;
    return CT_OK;
}

int ct_mlp_destroy(ct_mlp* mlp) {
    if (!mlp) return CT_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();   // launches on any stream may still use the buffers
    delete mlp;
    return CT_OK;
}

int ct_mlp_info(const ct_mlp* mlp, int64_t* n_params) {
    if (!mlp || !n_params) return CT_ERR_INVALID_ARG;
    *n_params = mlp->n_params;
    return CT_OK;
}

int ct_mlp_set_params(ct_mlp* mlp, const float* params, void* stream) {
    if (!mlp || !params) return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = (size_t)mlp->n_params * sizeof(float);
    int rc = err_of(hipMemcpyAsync(mlp->P, params, bytes, hipMemcpyDeviceToDevice, st));
    if (rc == CT_OK) rc = err_of(hipMemsetAsync(mlp->Mo, 0, bytes, st));
    if (rc == CT_OK) rc = err_of(hipMemsetAsync(mlp->Vo, 0, bytes, st));
    return rc != CT_OK ? rc : refresh(mlp, st);
}

int ct_mlp_get_params(const ct_mlp* mlp, float* params, void* stream) {
    if (!mlp || !params) return CT_ERR_INVALID_ARG;
    return err_of(hipMemcpyAsync(params, mlp->P, (size_t)mlp->n_params * sizeof(float), hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream));
}

int ct_mlp_get_grads(const ct_mlp* mlp, float* grads, void* stream) {
    if (!mlp || !grads) return CT_ERR_INVALID_ARG;
    return err_of(hipMemcpyAsync(grads, mlp->G, (size_t)mlp->n_params * sizeof(float), hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream));
}

int ct_mlp_noise(const ct_mlp* mlp, uint64_t seed, const int32_t* draw, int64_t rows, float* out, void* stream) {
    if (!mlp || rows < 0 || (rows > 0 && !out)) return CT_ERR_INVALID_ARG;
    if (rows == 0 || mlp->s.d_noise == 0) return CT_OK;
    const int64_t cnt = rows * (mlp->s.d_noise / 4);
    hipLaunchKernelGGL(noise_kernel, dim3(blocks(cnt, 256)), dim3(256), 0, (hipStream_t)stream, draw, rows,
                       mlp->s.d_noise, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), out);
    return err_of(hipGetLastError());
}

}  // extern "C"

namespace {

int forward_out(ct_mlp* mlp, const float* feats, int64_t n_feats, const int32_t* feat_of_row, const int32_t* draw,
                int64_t rows, uint64_t seed, float* Y, bool train, void* stream) {
    if (!mlp || rows < 0 || rows > mlp->rows_cap) return CT_ERR_INVALID_ARG;
    if (rows == 0) return CT_OK;
    if (!Y || (mlp->s.d_feat > 0 && (!feats || n_feats < 1))) return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    int rc = forward(mlp, feats, n_feats < 1 ? 1 : n_feats, feat_of_row, draw, 0, rows, seed, train, st);
    if (rc == CT_OK)
        rc = err_of(hipMemcpyAsync(Y, mlp->Y, (size_t)rows * mlp->s.d_out * sizeof(float), hipMemcpyDeviceToDevice,
                                   st));
    return rc;
}

}  // namespace

extern "C" {

int ct_mlp_forward(ct_mlp* mlp, const float* feats, int64_t n_feats, const int32_t* feat_of_row, const int32_t* draw,
                   int64_t rows, uint64_t seed, float* Y, void* stream) {
    return forward_out(mlp, feats, n_feats, feat_of_row, draw, rows, seed, Y, true, stream);
}

int ct_mlp_infer(ct_mlp* mlp, const float* feats, int64_t n_feats, const int32_t* feat_of_row, const int32_t* draw,
                 int64_t rows, uint64_t seed, float* Y, void* stream) {
    return forward_out(mlp, feats, n_feats, feat_of_row, draw, rows, seed, Y, false, stream);
}

int ct_mlp_backward(ct_mlp* mlp, const float* dY, int64_t rows, void* stream) {
    if (!mlp || !dY || rows <= 0 || rows % 64 != 0 || rows != mlp->fwd_rows) return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(out_grad_kernel, dim3(blocks(rows, 4)), dim3(256), 0, st, dY, (const float*)nullptr,
                       (const float*)nullptr, mlp->s.d_out, mlp->out_pad, rows, 1.f, mlp->GY, mlp->GYT, mlp->rows_cap,
                       (float*)nullptr);
    const int rc = err_of(hipGetLastError());
    return rc != CT_OK ? rc : backward(mlp, rows, st);
}

int ct_mlp_adam(ct_mlp* mlp, int64_t t, const ct_adam* adam_args, void* stream) {
    if (!mlp || t < 1 || !adam_ok(adam_args)) return CT_ERR_INVALID_ARG;
    return adam(mlp, t, adam_args, (hipStream_t)stream);
}

int ct_mlp_imle_step(ct_mlp* mlp, const float* feats, int64_t n_feats, const int32_t* feat_of_row,
                     const float* targets, const float* weights, int64_t rows, int32_t n_draws, uint64_t seed, int64_t t,
                     const ct_adam* adam_args, float* loss, int32_t* chosen, void* stream) {
    if (!mlp || !targets || rows <= 0 || rows % 64 != 0 || n_draws < 1 || t < 1 || !adam_ok(adam_args) ||
        rows * n_draws > mlp->rows_cap || (mlp->s.d_feat > 0 && (!feats || n_feats < 1)))
        return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nf = n_feats < 1 ? 1 : n_feats;
    int32_t* sel = chosen ? chosen : mlp->chosen;
    // 1. every draw, inference only; 2. the nearest draw per target, with
    // the squared-error gradient at its output and its input row for 3.
    int rc = forward(mlp, feats, nf, feat_of_row, nullptr, n_draws, rows * n_draws, seed, false, st);
    if (rc != CT_OK) return rc;
    SelectArgs sa{};
    sa.Y = mlp->Y;
    sa.T = targets;
    sa.W = weights;
    sa.d_out = mlp->s.d_out;
    sa.B = rows;
    sa.S = n_draws;
    sa.chosen = sel;
    sa.out_pad = mlp->out_pad;
    sa.scale = (float)(2.0 / ((double)rows * mlp->s.d_out));
    sa.GY = mlp->GY;
    sa.GYT = mlp->GYT;
    sa.ldt = mlp->rows_cap;
    sa.row_loss = mlp->row_loss;
    sa.in = input_args(mlp, feats, nf, feat_of_row, sel, 0, rows, seed, true);
    hipLaunchKernelGGL(imle_select_kernel, dim3((unsigned)rows), dim3(256), 0, st, sa);
    rc = err_of(hipGetLastError());
    // 3. the kept draws' hidden layers again, keeping activations (their
    // outputs are the selection forward's: same inputs, same weights)
    if (rc == CT_OK) rc = forward(mlp, feats, nf, feat_of_row, sel, 0, rows, seed, true, st, false, false);
    if (rc != CT_OK) return rc;
    // 4. backward (and the loss) and Adam
    if (rc == CT_OK) rc = backward(mlp, rows, st, loss, (float)(1.0 / ((double)rows * mlp->s.d_out)));
    if (rc == CT_OK) rc = adam(mlp, t, adam_args, st);
    return rc;
}

int ct_mlp_sample(ct_mlp* mlp, const float* feats, uint64_t seed, const float* mean, const float* std_,
                  const float* lo, const float* hi, const uint8_t* wrap, float* X, float* M, float* V, int64_t n,
                  int64_t ld, void* stream) {
    if (!mlp || n < 0 || ld < n || ld % 64 != 0 || up(n, 64) > mlp->rows_cap) return CT_ERR_INVALID_ARG;
    if (n == 0) return CT_OK;
    if (!mean || !std_ || !lo || !hi || !X || (mlp->s.d_feat > 0 && !feats)) return CT_ERR_INVALID_ARG;
    if (((uintptr_t)X % 256) || (M && (uintptr_t)M % 256) || (V && (uintptr_t)V % 256)) return CT_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    int rc = forward(mlp, feats, 1, nullptr, nullptr, 0, n, seed, false, st);
    if (rc != CT_OK) return rc;
    hipLaunchKernelGGL(sample_store_kernel, dim3(blocks(n, SEED_TILE)), dim3(256), 0, st, mlp->Y, mlp->s.d_out, n, mean,
                       std_, lo, hi, wrap, X, M, V, ld);
    return err_of(hipGetLastError());
}

}  // extern "C"
