// Learned reuse predictor (an extension of the reuse decision of Section 4,
// Alg. 1): label generation from the library's own FP32 derivation, and
// training with the library's own forward, backward and Adam kernels.
//
// Network: Linear(6,64) - ReLU - Linear(64,64) - ReLU - Linear(64,1) - sigmoid,
// parameters packed W1[64,6] b1 W2[64,64] b2 W3[1,64] b3.  Loss: mean BCE
// with positive-class weight w:  -(w y log p + (1-y) log(1-p)).
//
//   k_pred_fwdbwd   one thread per row: forward, dLoss/dlogit (/ rows),
//                   back-propagated dZ2, dZ1; stores X, H1, H2, dZ1, dZ2
//   k_pred_reduce   one thread per parameter: the batch sum of its gradient
//                   (fixed order, deterministic) and the batch loss
//   k_pred_adam     bias-corrected Adam step, then the BF16 inference copy
//   k_pred_infer    BF16 weights and activations, FP32 accumulate (the form
//                   the cache lookup uses)
//   k_pred_labels   compare every candidate's fresh derivation with its line
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "gsc_common.h"
#include "gsc_ctx.h"
#include "gsc_derive_mfma.h"
#include "gsc_pred_bf16.h"

namespace gsc {

namespace {

constexpr int NT = 256;
constexpr int P = GSC_PRED_NPARAMS;
constexpr int oW1 = 0, ob1 = 64 * 6, oW2 = ob1 + 64, ob2 = oW2 + 64 * 64, oW3 = ob2 + 64, ob3 = oW3 + 64;
constexpr int kMaxRows = 4096;

__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

__device__ __forceinline__ float softplus(float x) { return x > 0.f ? x + log1pf(expf(-x)) : log1pf(expf(x)); }

struct Work {
    float* X;    // [B][6]
    float* H1;   // [B][64]
    float* H2;   // [B][64]
    float* DZ1;  // [B][64]
    float* DZ2;  // [B][64]
    float* DL;   // [B] dLoss/dlogit (already divided by B)
    float* LS;   // [B] loss terms
};

__global__ __launch_bounds__(NT) void k_pred_fwdbwd(const float* __restrict__ w, const float* __restrict__ Xin,
                                                    const float* __restrict__ yf, const uint8_t* __restrict__ yb,
                                                    const int32_t* __restrict__ idx, int rows, float pos_weight,
                                                    Work wk) {
    const int r = (int)gtid();
    if (r >= rows) return;
    const int64_t src = idx ? idx[r] : r;
    float x[kPredIn];
#pragma unroll
    for (int i = 0; i < kPredIn; ++i) {
        x[i] = Xin[src * kPredIn + i];
        wk.X[(int64_t)r * kPredIn + i] = x[i];
    }
    const float y = yf ? yf[src] : (float)yb[src];
    float z1[kPredW], h1[kPredW];
#pragma unroll
    for (int j = 0; j < kPredW; ++j) {
        float a = w[ob1 + j];
#pragma unroll
        for (int i = 0; i < kPredIn; ++i) a = fmaf(w[oW1 + j * kPredIn + i], x[i], a);
        z1[j] = a;
        h1[j] = fmaxf(a, 0.f);
        wk.H1[(int64_t)r * kPredW + j] = h1[j];
    }
    float logit = w[ob3];
    float z2m[kPredW];  // sign mask of z2 (1 if positive)
    for (int j = 0; j < kPredW; ++j) {
        float a = w[ob2 + j];
#pragma unroll
        for (int i = 0; i < kPredW; ++i) a = fmaf(w[oW2 + j * kPredW + i], h1[i], a);
        float h2 = fmaxf(a, 0.f);
        z2m[j] = a > 0.f ? 1.f : 0.f;
        wk.H2[(int64_t)r * kPredW + j] = h2;
        logit = fmaf(w[oW3 + j], h2, logit);
    }
    const float p = 1.0f / (1.0f + expf(-logit));
    wk.LS[r] = pos_weight * y * softplus(-logit) + (1.0f - y) * softplus(logit);
    const float dl = (pos_weight * y * (p - 1.0f) + (1.0f - y) * p) / (float)rows;
    wk.DL[r] = dl;
    float dz2[kPredW];
#pragma unroll
    for (int j = 0; j < kPredW; ++j) {
        dz2[j] = dl * w[oW3 + j] * z2m[j];
        wk.DZ2[(int64_t)r * kPredW + j] = dz2[j];
    }
    for (int i = 0; i < kPredW; ++i) {
        float a = 0.f;
#pragma unroll
        for (int j = 0; j < kPredW; ++j) a = fmaf(w[oW2 + j * kPredW + i], dz2[j], a);
        wk.DZ1[(int64_t)r * kPredW + i] = z1[i] > 0.f ? a : 0.f;
    }
}

// grads[p] for every parameter, and grads[P] = mean loss.
__global__ __launch_bounds__(NT) void k_pred_reduce(Work wk, int rows, float* __restrict__ grads) {
    const int p = (int)gtid();
    if (p > P) return;
    float acc = 0.f;
    if (p == P) {
        for (int r = 0; r < rows; ++r) acc += wk.LS[r];
        grads[P] = acc / (float)rows;
        return;
    }
    if (p < ob1) {  // W1[j][i] = sum dz1[r][j] x[r][i]
        const int j = p / kPredIn, i = p % kPredIn;
        for (int r = 0; r < rows; ++r) acc = fmaf(wk.DZ1[(int64_t)r * kPredW + j], wk.X[(int64_t)r * kPredIn + i], acc);
    } else if (p < oW2) {
        const int j = p - ob1;
        for (int r = 0; r < rows; ++r) acc += wk.DZ1[(int64_t)r * kPredW + j];
    } else if (p < ob2) {
        const int j = (p - oW2) / kPredW, i = (p - oW2) % kPredW;
        for (int r = 0; r < rows; ++r) acc = fmaf(wk.DZ2[(int64_t)r * kPredW + j], wk.H1[(int64_t)r * kPredW + i], acc);
    } else if (p < oW3) {
        const int j = p - ob2;
        for (int r = 0; r < rows; ++r) acc += wk.DZ2[(int64_t)r * kPredW + j];
    } else if (p < ob3) {
        const int i = p - oW3;
        for (int r = 0; r < rows; ++r) acc = fmaf(wk.DL[r], wk.H2[(int64_t)r * kPredW + i], acc);
    } else {
        for (int r = 0; r < rows; ++r) acc += wk.DL[r];
    }
    grads[p] = acc;
}

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(NT) void k_pred_adam(float* __restrict__ w, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, float lr, float bc1,
                                                  float bc2, uint16_t* __restrict__ wbf, float* __restrict__ loss_acc,
                                                  int batches_done) {
    const int p = (int)gtid();
    if (p == 0 && loss_acc) *loss_acc += g[P];
    if (p >= P) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    const float nw = w[p] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[p] = nw;
    wbf[p] = to_bf16(nw);
    (void)batches_done;
}

__global__ __launch_bounds__(NT) void k_pred_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wbf) {
    const int p = (int)gtid();
    if (p < P) wbf[p] = to_bf16(w[p]);
}


// One candidate per lane; the loop is uniform per wave (the predictor runs
// on the whole wave).
__global__ __launch_bounds__(NT) void k_pred_infer(const uint16_t* __restrict__ wb, const float* __restrict__ w32,
                                                   const float* __restrict__ X, int64_t n, float* __restrict__ out) {
    __shared__ uint32_t s_h[NT / 64][kPredLdsWave];
    const int lane = threadIdx.x & 63;
    for (int64_t w0 = gtid() - lane; w0 < n; w0 += gstride()) {
        const int64_t r = w0 + lane;
        float x[kPredIn] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (r < n) {
#pragma unroll
            for (int i = 0; i < kPredIn; ++i) x[i] = X[r * kPredIn + i];
        }
        const float p = pred_prob_bf16_wave(wb, w32, x, s_h[threadIdx.x >> 6]);
        if (r < n) out[r] = p;
    }
}

__global__ __launch_bounds__(NT) void k_iota(int32_t* __restrict__ a, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) a[i] = (int32_t)i;
}

// Label per candidate: 1 iff its fresh derivation (scratch line i) differs
// from its cached one (line slot_of[anchor]) by more than the thresholds.
// Label of one reuse candidate: 1 (re-derive) when its cached Gaussians have
// drifted visibly from a fresh derivation at this frame.  The drift of one
// Gaussian is the largest of its opacity change, its colour change weighted by
// its opacity, and half the relative change of its covariance (the relative
// change of its footprint radius) weighted by its opacity; the anchor's drift
// (largest over its k Gaussians) times its projected footprint area in pixels,
// max(1, size^2) with size = 2^feature[5] the projected voxel size, must stay
// below the change of a 4x4-pixel patch by one 8-bit level (16/255).
__global__ __launch_bounds__(NT) void k_pred_labels(const int32_t* __restrict__ cand, const int32_t* __restrict__ slot_of,
                                                    const Counters* cnt, int k, const float* __restrict__ feat,
                                                    const float4* __restrict__ F0, const float4* __restrict__ F1,
                                                    const float4* __restrict__ F2, const float* __restrict__ F3,
                                                    const float4* __restrict__ C0, const float4* __restrict__ C1,
                                                    const float4* __restrict__ C2, const float* __restrict__ C3,
                                                    uint8_t* __restrict__ y) {
    const int64_t n = cnt->n_cand;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        const int64_t line = slot_of[cand[i]];
        if (line < 0) {
            y[i] = 1;
            continue;
        }
        float drift = 0.f;
        for (int j = 0; j < k; ++j) {
            const int64_t f = i * k + j, c = line * k + j;
            const float4 a0 = F0[f], a1 = F1[f], a2 = F2[f];
            const float a3 = F3[f];
            const float4 b0 = C0[c], b1 = C1[c], b2 = C2[c];
            const float b3 = C3[c];
            const float dc = fmaxf(fabsf(a2.z - b2.z), fmaxf(fabsf(a2.w - b2.w), fabsf(a3 - b3)));
            const float sa[6] = {a1.x, a1.y, a1.z, a1.w, a2.x, a2.y};
            const float sb[6] = {b1.x, b1.y, b1.z, b1.w, b2.x, b2.y};
            float dmax = 0.f, smax = 0.f;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                dmax = fmaxf(dmax, fabsf(sa[q] - sb[q]));
                smax = fmaxf(smax, fabsf(sa[q]));
            }
            const float geo = smax > 0.f ? dmax / smax : (dmax > 0.f ? INFINITY : 0.f);
            const float am = fmaxf(fabsf(a0.w), fabsf(b0.w));
            drift = fmaxf(drift, fmaxf(fabsf(a0.w - b0.w), am * fmaxf(dc, 0.5f * geo)));
        }
        const float size = exp2f(feat[i * kPredIn + 5]);
        y[i] = drift * fmaxf(1.f, size * size) > 16.0f / 255.0f ? 1 : 0;
    }
}

int fail(gsc_ctx* c, int code, const char* msg) {
    c->err = msg;
    return code;
}

hipError_t ensure_pred(gsc_ctx* c) {
    if (c->pred_w) return hipSuccess;
    size_t b = 0;
    hipError_t e;
    if ((e = dalloc(c->pmem, b, &c->pred_w, P)) != hipSuccess || (e = dalloc(c->pmem, b, &c->pred_wbf, P)) != hipSuccess ||
        (e = dalloc(c->pmem, b, &c->pred_m, P)) != hipSuccess || (e = dalloc(c->pmem, b, &c->pred_v, P)) != hipSuccess ||
        (e = dalloc(c->pmem, b, &c->pred_g, P + 1)) != hipSuccess || (e = dalloc(c->pmem, b, &c->pred_loss, 1)) != hipSuccess ||
        (e = dalloc(c->pmem, b, &c->pred_work, (size_t)kMaxRows * (kPredIn + 4 * kPredW + 2))) != hipSuccess ||
        (e = dalloc(c->pmem, b, &c->pred_idx, kMaxRows)) != hipSuccess) {
        return e;
    }
    return hipSuccess;
}

Work work_of(gsc_ctx* c) {
    Work w;
    float* p = c->pred_work;
    w.X = p; p += (size_t)kMaxRows * kPredIn;
    w.H1 = p; p += (size_t)kMaxRows * kPredW;
    w.H2 = p; p += (size_t)kMaxRows * kPredW;
    w.DZ1 = p; p += (size_t)kMaxRows * kPredW;
    w.DZ2 = p; p += (size_t)kMaxRows * kPredW;
    w.DL = p; p += kMaxRows;
    w.LS = p;
    return w;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, kGridBlocks)); }

}  // namespace

void pred_free(gsc_ctx* c) {
    free_labels(c);
    if (c->pmem.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    c->pmem.release();
    c->pred_w = nullptr;
    c->pred_wbf = nullptr;
    c->pred_m = c->pred_v = c->pred_g = c->pred_loss = c->pred_work = nullptr;
    c->pred_idx = nullptr;
    c->pred_loaded = false;
}

}  // namespace gsc

using namespace gsc;

extern "C" {

int gsc_predictor_load(gsc_ctx* c, const float* params, int64_t n) {
    if (!c || !params) return c ? fail(c, GSC_E_INVALID_ARG, "gsc_predictor_load: null argument") : GSC_E_INVALID_ARG;
    if (n != P) return fail(c, GSC_E_INVALID_ARG, "gsc_predictor_load: wrong parameter count");
    if (ensure_pred(c) != hipSuccess) return fail(c, GSC_E_OOM, "gsc_predictor_load: device allocation");
    if (hipMemcpyAsync(c->pred_w, params, P * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemsetAsync(c->pred_m, 0, P * 4, c->stream) != hipSuccess ||
        hipMemsetAsync(c->pred_v, 0, P * 4, c->stream) != hipSuccess)
        return fail(c, GSC_E_HIP, "gsc_predictor_load: copy failed");
    hipLaunchKernelGGL(k_pred_to_bf16, dim3(blocks_for(P)), dim3(NT), 0, c->stream, c->pred_w, c->pred_wbf);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, GSC_E_HIP, "gsc_predictor_load: sync failed");
    c->pred_step = 0;
    c->pred_loaded = true;
    return GSC_OK;
}

int gsc_predictor_get(gsc_ctx* c, float* params, int64_t n) {
    if (!c || !params) return c ? fail(c, GSC_E_INVALID_ARG, "gsc_predictor_get: null argument") : GSC_E_INVALID_ARG;
    if (n != P) return fail(c, GSC_E_INVALID_ARG, "gsc_predictor_get: wrong parameter count");
    if (!c->pred_loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_predictor_get: no predictor loaded");
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(params, c->pred_w, P * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, GSC_E_HIP, "gsc_predictor_get: copy failed");
    return GSC_OK;
}

int gsc_predictor_collect(gsc_ctx* c, int enable) {
    if (!c) return GSC_E_INVALID_ARG;
    c->collect_features = enable ? 1 : 0;
    return GSC_OK;
}

int gsc_predictor_labels(gsc_ctx* c, float* X_out, uint8_t* y_out, int32_t* ids_out, int64_t cap, int64_t* n) {
    if (!c || !n) return c ? fail(c, GSC_E_INVALID_ARG, "gsc_predictor_labels: null argument") : GSC_E_INVALID_ARG;
    if (cap > 0 && (!X_out || !y_out)) return fail(c, GSC_E_INVALID_ARG, "gsc_predictor_labels: null output");
    if (!c->loaded || !c->derived || !c->collect_features)
        return fail(c, GSC_E_NOT_LOADED, "gsc_predictor_labels: needs a gsc_derive with collection enabled");
    if (!(c->cfg.flags & GSC_FLAG_REUSE) || c->nviews != 1)
        return fail(c, GSC_E_INVALID_ARG, "gsc_predictor_labels: needs reuse on and de-redundancy on");
    View& v = c->view[0];
    const Scene& sc = c->scene;
    hipStream_t st = c->stream;
    const int64_t E = sc.n * sc.k;
    if (c->lab_entries < E) {  // scratch lines for fresh derivations of the candidates
        free_labels(c);
        size_t b = 0;
        hipError_t e;
        if ((e = dalloc(c->lmem, b, &c->lab_L0, E)) != hipSuccess || (e = dalloc(c->lmem, b, &c->lab_L1, E)) != hipSuccess ||
            (e = dalloc(c->lmem, b, &c->lab_L2, E)) != hipSuccess || (e = dalloc(c->lmem, b, &c->lab_L3, E)) != hipSuccess ||
            (e = dalloc(c->lmem, b, &c->lab_iota, sc.n)) != hipSuccess || (e = dalloc(c->lmem, b, &c->lab_y, sc.n)) != hipSuccess) {
            free_labels(c);
            return fail(c, GSC_E_OOM, "gsc_predictor_labels: device allocation");
        }
        c->lab_entries = E;
        hipLaunchKernelGGL(k_iota, dim3(blocks_for(sc.n)), dim3(NT), 0, st, c->lab_iota, sc.n);
    }
    // derive every candidate again with this frame's unified camera, FP32
    MfmaDeriveArgs m;
    m.posr = sc.posr; m.feat = sc.feat; m.scale = sc.scale; m.offsets = sc.offsets; m.k = sc.k;
    m.visible = v.cand_id; m.misses = c->lab_iota; m.vslot = c->lab_iota;
    m.L0 = c->lab_L0; m.L1 = c->lab_L1; m.L2 = c->lab_L2; m.L3 = c->lab_L3; m.line_mask = nullptr;
    for (int i = 0; i < 3; ++i) m.cam_pos[i] = (float)c->unified.pos[i];
    m.inv_dist_unit = sc.dist_unit > 0.f ? 1.0f / sc.dist_unit : 0.f;
    m.n_miss = &v.cnt->n_cand; m.mode = GSC_PREC_F32;
    m.fr.l1_f32 = sc.fr_l1_f32; m.fr.l2_f32 = sc.fr_l2_f32; m.fr.l1_bf16 = sc.fr_l1_bf16;
    m.fr.l2_bf16 = sc.fr_l2_bf16; m.fr.l1_fp8 = sc.fr_l1_fp8; m.fr.l2_fp8 = sc.fr_l2_fp8;
    m.fr.b1 = sc.fr_b1; m.fr.b2 = sc.fr_b2; m.fr.s1 = sc.fr_s1; m.fr.s2 = sc.fr_s2;
    m.fr.n_at = sc.n_at; m.fr.n_ct = sc.n_ct; m.fr.n_vt = sc.n_vt;
    if (derive_mfma(m, sc.n, st) != hipSuccess) return fail(c, GSC_E_HIP, "gsc_predictor_labels: derive failed");
    hipLaunchKernelGGL(k_pred_labels, dim3(blocks_for(sc.n)), dim3(NT), 0, st, v.cand_id, v.slot_of, v.cnt, sc.k,
                       v.cand_feat, c->lab_L0, c->lab_L1, c->lab_L2, c->lab_L3, v.L0, v.L1, v.L2, v.L3, c->lab_y);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(c, GSC_E_HIP, "gsc_predictor_labels: kernels failed");
    Counters k;
    if (hipMemcpy(&k, v.cnt, sizeof(k), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, GSC_E_HIP, "gsc_predictor_labels: copy failed");
    *n = k.n_cand;
    const int64_t m_out = std::min<int64_t>(cap, k.n_cand);
    if (m_out > 0 && (hipMemcpy(X_out, v.cand_feat, m_out * kPredIn * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                      hipMemcpy(y_out, c->lab_y, m_out, hipMemcpyDeviceToHost) != hipSuccess))
        return fail(c, GSC_E_HIP, "gsc_predictor_labels: copy failed");
    if (m_out > 0 && ids_out && hipMemcpy(ids_out, v.cand_id, m_out * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, GSC_E_HIP, "gsc_predictor_labels: copy failed");
    return GSC_OK;
}

int gsc_predictor_grad(gsc_ctx* c, const float* X, const float* y, int64_t n, float pos_weight, float* grads_out,
                       float* loss_out) {
    if (!c || !X || !y || !grads_out) return c ? fail(c, GSC_E_INVALID_ARG, "gsc_predictor_grad: null argument")
                                               : GSC_E_INVALID_ARG;
    if (n < 1 || n > kMaxRows) return fail(c, GSC_E_INVALID_ARG, "gsc_predictor_grad: n must be in [1, 4096]");
    if (!c->pred_loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_predictor_grad: no predictor loaded");
    Work wk = work_of(c);
    hipLaunchKernelGGL(k_pred_fwdbwd, dim3(blocks_for(n)), dim3(NT), 0, c->stream, c->pred_w, X, y, nullptr, nullptr,
                       (int)n, pos_weight, wk);
    hipLaunchKernelGGL(k_pred_reduce, dim3(blocks_for(P + 1)), dim3(NT), 0, c->stream, wk, (int)n, c->pred_g);
    std::vector<float> g(P + 1);
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(g.data(), c->pred_g, (P + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, GSC_E_HIP, "gsc_predictor_grad: kernels failed");
    std::memcpy(grads_out, g.data(), P * 4);
    if (loss_out) *loss_out = g[P];
    return GSC_OK;
}

int gsc_predictor_train(gsc_ctx* c, const float* X, const uint8_t* y, int64_t n, int32_t batch, int32_t epochs,
                        float lr, float pos_weight, uint64_t seed, float* loss_out) {
    if (!c || !X || !y) return c ? fail(c, GSC_E_INVALID_ARG, "gsc_predictor_train: null argument") : GSC_E_INVALID_ARG;
    if (n < 1 || batch < 1 || batch > kMaxRows || epochs < 1 || !(lr > 0.f))
        return fail(c, GSC_E_INVALID_ARG, "gsc_predictor_train: bad sizes");
    if (!c->pred_loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_predictor_train: load initial weights first");
    hipStream_t st = c->stream;
    float* dX = nullptr;
    uint8_t* dy = nullptr;
    int32_t* dperm = nullptr;
    if (hipMalloc((void**)&dX, n * kPredIn * 4) != hipSuccess || hipMalloc((void**)&dy, n) != hipSuccess ||
        hipMalloc((void**)&dperm, n * 4) != hipSuccess) {
        (void)hipFree(dX); (void)hipFree(dy); (void)hipFree(dperm);
        return fail(c, GSC_E_OOM, "gsc_predictor_train: device allocation");
    }
    int rc = GSC_OK;
    std::vector<int32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::mt19937_64 rng(seed);
    Work wk = work_of(c);
    if (hipMemcpyAsync(dX, X, n * kPredIn * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dy, y, n, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = fail(c, GSC_E_HIP, "gsc_predictor_train: upload failed");
    for (int ep = 0; ep < epochs && rc == GSC_OK; ++ep) {
        std::shuffle(perm.begin(), perm.end(), rng);
        if (hipMemcpyAsync(dperm, perm.data(), n * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemsetAsync(c->pred_loss, 0, 4, st) != hipSuccess) {
            rc = fail(c, GSC_E_HIP, "gsc_predictor_train: upload failed");
            break;
        }
        int nb = 0;
        for (int64_t b0 = 0; b0 < n; b0 += batch, ++nb) {
            const int rows = (int)std::min<int64_t>(batch, n - b0);
            hipLaunchKernelGGL(k_pred_fwdbwd, dim3(blocks_for(rows)), dim3(NT), 0, st, c->pred_w, dX, nullptr, dy,
                               dperm + b0, rows, pos_weight, wk);
            hipLaunchKernelGGL(k_pred_reduce, dim3(blocks_for(P + 1)), dim3(NT), 0, st, wk, rows, c->pred_g);
            c->pred_step += 1;
            const float bc1 = 1.0f - (float)std::pow(0.9, c->pred_step);
            const float bc2 = 1.0f - (float)std::pow(0.999, c->pred_step);
            hipLaunchKernelGGL(k_pred_adam, dim3(blocks_for(P)), dim3(NT), 0, st, c->pred_w, c->pred_g, c->pred_m,
                               c->pred_v, lr, bc1, bc2, c->pred_wbf, c->pred_loss, nb);
        }
        float lsum = 0.f;
        if (hipMemcpyAsync(&lsum, c->pred_loss, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(c, GSC_E_HIP, "gsc_predictor_train: training kernels failed");
            break;
        }
        if (loss_out) loss_out[ep] = lsum / (float)nb;
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(dX);
    (void)hipFree(dy);
    (void)hipFree(dperm);
    return rc;
}

int gsc_predictor_infer(gsc_ctx* c, const float* X, int64_t n, float* p_out) {
    if (!c || !X || !p_out) return c ? fail(c, GSC_E_INVALID_ARG, "gsc_predictor_infer: null argument")
                                     : GSC_E_INVALID_ARG;
    if (n < 0) return fail(c, GSC_E_INVALID_ARG, "gsc_predictor_infer: negative n");
    if (!c->pred_loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_predictor_infer: no predictor loaded");
    if (n == 0) return GSC_OK;
    hipLaunchKernelGGL(k_pred_infer, dim3(blocks_for(n)), dim3(NT), 0, c->stream, c->pred_wbf, c->pred_w, X, n, p_out);
    if (hipGetLastError() != hipSuccess) return fail(c, GSC_E_HIP, "gsc_predictor_infer: launch failed");
    return GSC_OK;
}

}  // extern "C"
