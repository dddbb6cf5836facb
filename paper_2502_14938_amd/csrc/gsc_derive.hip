// Derive stage of one frame of one viewer (Section 4, Alg. 1):
//   anchor indexing + filtering  -> k_select_flags + compaction (X_t, ascending)
//   cache scheduling             -> k_cache_* (invalidate at the reuse depth,
//                                   hit/miss, learned staleness, slot
//                                   allocation, eviction of outdated lines)
//   decode new anchors           -> k_derive_f32 / derive_mfma (eq. 3, eq. 2)
//   configure the cache depth    -> k_depth_update (eq. 4, linear guide)
//   update the render buffer     -> k_compose_* (opacity mask, Section 6)
// Every count stays on the device (Counters); the host only enqueues.
#include <cmath>

#include "gsc_common.h"
#include "gsc_derive_mfma.h"

namespace gsc {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// ------------------------------------------------------------- selection
// Keep anchor a iff (level 0 or |x - p_u| <= d_ref 2^-level) and its bounding
// sphere is not wholly outside any unified-frustum plane (4 sides + near).
__global__ __launch_bounds__(NT) void k_select_flags(const float4* __restrict__ posr, const uint8_t* __restrict__ level,
                                                     int64_t n, DeriveCam cam, uint32_t* __restrict__ flags) {
    for (int64_t a = gtid(); a < n; a += gstride()) {
        float4 p = posr[a];
        int l = level[a];
        bool keep = true;
        if (l != 0) {
            float vx = p.x - cam.pos[0], vy = p.y - cam.pos[1], vz = p.z - cam.pos[2];
            float lim = ldexpf(cam.d_ref, -l);
            keep = vx * vx + vy * vy + vz * vz <= lim * lim;
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            float s = cam.planes[i][0] * p.x + cam.planes[i][1] * p.y + cam.planes[i][2] * p.z + cam.planes[i][3];
            keep = keep && (s >= -p.w);
        }
        flags[a] = keep ? 1u : 0u;
    }
}

// out[scan[i]] = i for flagged i (ascending).
__global__ __launch_bounds__(NT) void k_compact_ids(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                                                    int64_t n, const int32_t* n_dev, int32_t* __restrict__ out) {
    int64_t m = n_dev ? *n_dev : n;
    for (int64_t i = gtid(); i < m; i += gstride())
        if (flags[i]) out[pos[i]] = (int32_t)i;
}

// ------------------------------------------------------------- cache

// Alg. 1: invalidate every line whose age exceeds the current depth.
__global__ __launch_bounds__(NT) void k_cache_invalidate(int32_t* __restrict__ line_anchor, const int32_t* __restrict__ tau,
                                                         int32_t* __restrict__ slot_of, int64_t C, int32_t t,
                                                         Counters* cnt) {
    int32_t d = cnt->depth;
    for (int64_t s = gtid(); s < C; s += gstride()) {
        int32_t a = line_anchor[s];
        if (a >= 0 && t - tau[s] > d) {
            slot_of[a] = -1;
            line_anchor[s] = -1;
        }
    }
}

// Learned staleness (reuse predictor): features of one candidate.
__device__ __forceinline__ void reuse_features(float4 p, int lvl, int lmax, const float* sc, const float* pu_now,
                                               const float* pu_then, int age, int dmax, float fx, float* f) {
    float vn[3] = {p.x - pu_now[0], p.y - pu_now[1], p.z - pu_now[2]};
    float vt[3] = {p.x - pu_then[0], p.y - pu_then[1], p.z - pu_then[2]};
    float dn = sqrtf(vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]);
    float dt = sqrtf(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
    float c = (vn[0] * vt[0] + vn[1] * vt[1] + vn[2] * vt[2]) / (dn * dt);
    float du[3] = {pu_now[0] - pu_then[0], pu_now[1] - pu_then[1], pu_now[2] - pu_then[2]};
    float smax = fmaxf(sc[0], fmaxf(sc[1], sc[2]));
    f[0] = 1.0f - c;
    f[1] = logf(dn / dt);
    f[2] = (float)age / (float)dmax;
    f[3] = (float)lvl / (float)(lmax > 0 ? lmax : 1);
    f[4] = sqrtf(du[0] * du[0] + du[1] * du[1] + du[2] * du[2]) / dn;
    f[5] = log2f(smax * fx / dn);
}

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// p(stale) with BF16 weights and activations, FP32 accumulation.
__device__ float pred_prob_bf16(const uint16_t* __restrict__ wb, const float* __restrict__ w32, const float* f) {
    // layout: W1[64*6] b1[64] W2[64*64] b2[64] W3[64] b3[1]
    const int oW1 = 0, ob1 = 64 * 6, oW2 = ob1 + 64, ob2 = oW2 + 64 * 64, oW3 = ob2 + 64, ob3 = oW3 + 64;
    float x[kPredIn];
#pragma unroll
    for (int i = 0; i < kPredIn; ++i) x[i] = bf16_round(f[i]);
    float h1[kPredW];
#pragma unroll
    for (int r = 0; r < kPredW; ++r) {
        float acc = 0.f;
#pragma unroll
        for (int c = 0; c < kPredIn; ++c) acc = fmaf(bf16_to_f(wb[oW1 + r * kPredIn + c]), x[c], acc);
        acc += w32[ob1 + r];
        h1[r] = bf16_round(fmaxf(acc, 0.f));
    }
    float logit = w32[ob3];
    for (int r = 0; r < kPredW; ++r) {
        float acc = 0.f;
#pragma unroll
        for (int c = 0; c < kPredW; ++c) acc = fmaf(bf16_to_f(wb[oW2 + r * kPredW + c]), h1[c], acc);
        acc += w32[ob2 + r];
        float h2 = bf16_round(fmaxf(acc, 0.f));
        logit = fmaf(bf16_to_f(wb[oW3 + r]), h2, logit);
    }
    return 1.0f / (1.0f + expf(-logit));
}

struct LookupArgs {
    const int32_t* visible;
    const int32_t* slot_of;
    int32_t* line_last;
    const int32_t* line_tau;
    uint32_t* miss_flag;   // [n_visible]
    int32_t t;
    int32_t reuse;
    int32_t predictor;
    float thr;
    const float4* posr;
    const uint8_t* level;
    const float* scale;
    const float* pu_hist;
    int32_t lmax, dmax;
    DeriveCam cam;
    const uint16_t* pred_wbf;
    const float* pred_w32;
    float* cand_feat;      // optional: features of candidates (for label collection)
    int32_t* cand_id;
    Counters* cnt;
};

// Hit iff the anchor still owns a line (after invalidation every owned line
// has 1 <= t - tau <= d_t), reuse is on and the predictor does not flag it.
// Every visible owned line is stamped last_used = t.
__global__ __launch_bounds__(NT) void k_cache_lookup(LookupArgs a) {
    int32_t nv = a.cnt->n_visible;
    for (int64_t i = gtid(); i < nv; i += gstride()) {
        int32_t aid = a.visible[i];
        int32_t s = a.slot_of[aid];
        bool hit = s >= 0 && a.reuse;
        if (s >= 0) a.line_last[s] = a.t;
        if (hit && (a.predictor || a.cand_feat)) {
            float f[kPredIn];
            int32_t tau = a.line_tau[s];
            reuse_features(a.posr[aid], a.level[aid], a.lmax, a.scale + 6 * (int64_t)aid, a.cam.pos,
                           a.pu_hist + 4 * (tau & 63), a.t - tau, a.dmax, a.cam.fx, f);
            if (a.cand_feat) {
                int32_t c = atomicAdd(&a.cnt->n_cand, 1);
                for (int q = 0; q < kPredIn; ++q) a.cand_feat[(int64_t)c * kPredIn + q] = f[q];
                a.cand_id[c] = aid;
            }
            if (a.predictor && pred_prob_bf16(a.pred_wbf, a.pred_w32, f) > a.thr) hit = false;
        }
        a.miss_flag[i] = hit ? 0u : 1u;
    }
}

// need[j] = 1 iff miss j (visible position misses[j]) owns no line.
__global__ __launch_bounds__(NT) void k_need_flags(const int32_t* __restrict__ misses, const int32_t* __restrict__ visible,
                                                   const int32_t* __restrict__ slot_of, Counters* cnt,
                                                   uint32_t* __restrict__ need) {
    int32_t nm = cnt->n_miss;
    for (int64_t j = gtid(); j < nm; j += gstride()) need[j] = slot_of[visible[misses[j]]] < 0 ? 1u : 0u;
}

__global__ __launch_bounds__(NT) void k_free_flags(const int32_t* __restrict__ line_anchor, int64_t C,
                                                   uint32_t* __restrict__ flags) {
    for (int64_t s = gtid(); s < C; s += gstride()) flags[s] = line_anchor[s] < 0 ? 1u : 0u;
}

// Eviction plan: lines not visible now (last_used < t) are candidates; take
// them in ascending (last_used, anchor).  last_used of a surviving line lies
// in [t - d_max, t - 1], so a d_max-bin histogram finds the threshold bin.
__global__ __launch_bounds__(NT) void k_evict_hist(const int32_t* __restrict__ line_anchor,
                                                   const int32_t* __restrict__ line_last, int64_t C, int32_t t,
                                                   int32_t dmax, Counters* cnt, uint32_t* __restrict__ hist) {
    if (cnt->n_need - cnt->n_free <= 0) return;
    __shared__ uint32_t h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t s = gtid(); s < C; s += gstride()) {
        int32_t lu = line_last[s];
        if (line_anchor[s] >= 0 && lu < t) {
            int b = lu - (t - dmax);
            b = b < 0 ? 0 : b;
            atomicAdd(&h[b], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < dmax && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_evict_plan(const uint32_t* __restrict__ hist, int32_t t, int32_t dmax, Counters* cnt,
                             int32_t* scan_n, int64_t n_anchor) {
    int32_t shortfall = cnt->n_need - cnt->n_free;
    cnt->evict_short = shortfall > 0 ? shortfall : 0;
    cnt->n_evict = 0;
    *scan_n = 0;
    if (shortfall <= 0) return;
    int32_t acc = 0;
    for (int b = 0; b < dmax; ++b) {
        int32_t h = (int32_t)hist[b];
        if (acc + h >= shortfall) {
            cnt->evict_thr = (t - dmax) + b;
            cnt->evict_left = shortfall - acc;
            cnt->n_evict = shortfall;
            *scan_n = (int32_t)n_anchor;
            return;
        }
        acc += h;
    }
    cnt->overflow |= 2;  // fewer evictable lines than needed
    cnt->evict_thr = t;  // evict every candidate; the frame is marked overflowed
    cnt->evict_left = 0;
    cnt->n_evict = acc;
}

// Anchors (ascending id) whose line sits in the threshold bin.
__global__ __launch_bounds__(NT) void k_evict_thr_flags(const int32_t* __restrict__ slot_of,
                                                        const int32_t* __restrict__ line_last, const int32_t* scan_n,
                                                        Counters* cnt, uint32_t* __restrict__ flags) {
    int64_t n = *scan_n;
    int32_t thr = cnt->evict_thr;
    for (int64_t a = gtid(); a < n; a += gstride()) {
        int32_t s = slot_of[a];
        flags[a] = (s >= 0 && line_last[s] == thr) ? 1u : 0u;
    }
}

__global__ __launch_bounds__(NT) void k_evict_apply(int32_t* __restrict__ line_anchor, const int32_t* __restrict__ line_last,
                                                    int32_t* __restrict__ slot_of, const uint32_t* __restrict__ rank,
                                                    int64_t C, int32_t t, Counters* cnt) {
    if (cnt->evict_short <= 0) return;
    int32_t thr = cnt->evict_thr, left = cnt->evict_left;
    for (int64_t s = gtid(); s < C; s += gstride()) {
        int32_t a = line_anchor[s];
        int32_t lu = line_last[s];
        if (a < 0 || lu >= t) continue;
        if (lu < thr || (lu == thr && (int32_t)rank[a] < left)) {
            slot_of[a] = -1;
            line_anchor[s] = -1;
        }
    }
}

// Misses without a line take free lines in ascending order; every miss is
// re-derived now (tau = t).
__global__ __launch_bounds__(NT) void k_assign(const int32_t* __restrict__ misses, const int32_t* __restrict__ visible,
                                               int32_t* __restrict__ slot_of, int32_t* __restrict__ line_anchor,
                                               int32_t* __restrict__ line_tau, int32_t* __restrict__ line_last,
                                               const uint32_t* __restrict__ need, const uint32_t* __restrict__ need_rank,
                                               const int32_t* __restrict__ free_list, int32_t t, int64_t C,
                                               Counters* cnt) {
    int32_t nm = cnt->n_miss;
    for (int64_t j = gtid(); j < nm; j += gstride()) {
        int32_t aid = visible[misses[j]];
        int32_t s;
        if (need[j]) {
            uint32_t r = need_rank[j];
            if ((int64_t)r >= C || r >= (uint32_t)max(cnt->n_free + cnt->n_evict, 0)) {
                atomicOr(&cnt->overflow, 2);
                continue;
            }
            s = free_list[r];
            slot_of[aid] = s;
            line_anchor[s] = aid;
            line_last[s] = t;
        } else {
            s = slot_of[aid];
        }
        line_tau[s] = t;
    }
}

__global__ __launch_bounds__(NT) void k_vslot(const int32_t* __restrict__ visible, const int32_t* __restrict__ slot_of,
                                              int32_t* __restrict__ vslot, Counters* cnt) {
    int32_t nv = cnt->n_visible;
    for (int64_t i = gtid(); i < nv; i += gstride()) vslot[i] = slot_of[visible[i]];
}

// No-cache schedule: every visible anchor is a miss derived into line i.
__global__ __launch_bounds__(NT) void k_nocache(int32_t* __restrict__ misses, int32_t* __restrict__ vslot, Counters* cnt) {
    int32_t nv = cnt->n_visible;
    if (gtid() == 0) cnt->n_miss = nv;
    for (int64_t i = gtid(); i < nv; i += gstride()) {
        misses[i] = (int32_t)i;
        vslot[i] = (int32_t)i;
    }
}

// Eq. 4 with the linear guiding function on the update (miss) rate.
__global__ void k_depth_update(Counters* cnt, int32_t dmax, int32_t guide) {
    int32_t nx = cnt->n_visible, nm = cnt->n_miss;
    cnt->depth_used = cnt->depth;
    if (guide == GSC_GUIDE_FIXED) {
        cnt->depth = dmax;
        return;
    }
    if (nx <= 0) return;
    int64_t d = (2ll * dmax * (nx - nm) + nx) / (2ll * nx);
    cnt->depth = (int32_t)(d < 1 ? 1 : (d > dmax ? dmax : d));
}

__global__ void k_frame_begin(Counters* cnt) {
    cnt->n_cand = 0;
    cnt->overflow = 0;
    cnt->n_evict = 0;
    cnt->evict_short = 0;
}

__global__ void k_evict_freescan_n(const Counters* cnt, int32_t* scan_n, int64_t C) {
    *scan_n = cnt->evict_short > 0 ? (int32_t)C : 0;
}

__global__ __launch_bounds__(NT) void k_free_flags_n(const int32_t* __restrict__ line_anchor, const int32_t* n_dev,
                                                     uint32_t* __restrict__ flags) {
    int64_t C = *n_dev;
    for (int64_t s = gtid(); s < C; s += gstride()) flags[s] = line_anchor[s] < 0 ? 1u : 0u;
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

__global__ void k_store_pu(float* pu_hist, int32_t t, DeriveCam cam) {
    if (threadIdx.x < 3) pu_hist[4 * (t & 63) + threadIdx.x] = cam.pos[threadIdx.x];
}

// ---------------------------------------------------------- derivation FP32
// One thread per missed anchor: the three heads' hidden layers (F+3 -> H)
// are computed once per anchor and shared by its k Gaussians (the anchor row
// is loaded once, no per-offset copies), then each Gaussian's 11 outputs are
// produced and written straight into the cache line arrays.
struct DeriveK {
    const float4* posr;
    const float* feat;
    const float* scale;
    const float* offsets;
    const float* w;  // packed fp32 weights
    WeightLayout L;
    int k;
    const int32_t* visible;
    const int32_t* misses;
    const int32_t* vslot;
    float4* L0;
    float4* L1;
    float4* L2;
    float* L3;
    DeriveCam cam;
    Counters* cnt;
};

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

__device__ __forceinline__ void write_gaussian(const DeriveK& a, int64_t e, float4 x, const float* sc, const float* O,
                                               float oa, const float* oc, const float* os) {
    float alpha = tanhf(oa);
    float s0 = sc[3] * sigm(os[0]), s1 = sc[4] * sigm(os[1]), s2 = sc[5] * sigm(os[2]);
    float qw = os[3], qx = os[4], qy = os[5], qz = os[6];
    float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    if (qn > 0.f) {
        float inv = 1.0f / qn;
        qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    } else {
        qw = 1.f; qx = qy = qz = 0.f;
    }
    float R[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
                     {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
                     {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
    float v[3] = {s0 * s0, s1 * s1, s2 * s2};
    float S[6];
    int idx = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = r; c < 3; ++c) S[idx++] = R[r][0] * v[0] * R[c][0] + R[r][1] * v[1] * R[c][1] + R[r][2] * v[2] * R[c][2];
    float mx = x.x + sc[0] * O[0], my = x.y + sc[1] * O[1], mz = x.z + sc[2] * O[2];
    a.L0[e] = make_float4(mx, my, mz, alpha);
    a.L1[e] = make_float4(S[0], S[1], S[2], S[3]);
    a.L2[e] = make_float4(S[4], S[5], sigm(oc[0]), sigm(oc[1]));
    a.L3[e] = sigm(oc[2]);
}

__global__ __launch_bounds__(NT) void k_derive_f32(DeriveK a) {
    const float* __restrict__ w = a.w;
    int32_t nm = a.cnt->n_miss;
    for (int64_t j = gtid(); j < nm; j += gstride()) {
        int32_t pos = a.misses[j];
        int32_t aid = a.visible[pos];
        int64_t line = a.vslot[pos];
        if (line < 0) continue;  // no line (cache capacity exceeded this frame)
        float4 x = a.posr[aid];
        float z[kF + 3];
        const float4* f4 = reinterpret_cast<const float4*>(a.feat + (int64_t)aid * kF);
#pragma unroll
        for (int q = 0; q < kF / 4; ++q) {
            float4 v = f4[q];
            z[4 * q] = v.x; z[4 * q + 1] = v.y; z[4 * q + 2] = v.z; z[4 * q + 3] = v.w;
        }
        float vx = x.x - a.cam.pos[0], vy = x.y - a.cam.pos[1], vz = x.z - a.cam.pos[2];
        float inv = 1.0f / sqrtf(vx * vx + vy * vy + vz * vz);
        z[kF] = vx * inv; z[kF + 1] = vy * inv; z[kF + 2] = vz * inv;
        float h[3][kH];
#pragma unroll
        for (int hd = 0; hd < 3; ++hd) {
            const float* W1 = w + a.L.W1[hd];
            const float* b1 = w + a.L.b1[hd];
#pragma unroll
            for (int r = 0; r < kH; ++r) {
                float acc = b1[r];
#pragma unroll
                for (int c = 0; c < kF + 3; ++c) acc = fmaf(W1[r * (kF + 3) + c], z[c], acc);
                h[hd][r] = fmaxf(acc, 0.f);
            }
        }
        float sc[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) sc[q] = a.scale[(int64_t)aid * 6 + q];
        const float* W2a = w + a.L.W2[0]; const float* b2a = w + a.L.b2[0];
        const float* W2c = w + a.L.W2[1]; const float* b2c = w + a.L.b2[1];
        const float* W2s = w + a.L.W2[2]; const float* b2s = w + a.L.b2[2];
        for (int g = 0; g < a.k; ++g) {
            float oa = b2a[g];
#pragma unroll
            for (int c = 0; c < kH; ++c) oa = fmaf(W2a[g * kH + c], h[0][c], oa);
            float oc[3], os[7];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                float acc = b2c[3 * g + q];
#pragma unroll
                for (int c = 0; c < kH; ++c) acc = fmaf(W2c[(3 * g + q) * kH + c], h[1][c], acc);
                oc[q] = acc;
            }
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                float acc = b2s[7 * g + q];
#pragma unroll
                for (int c = 0; c < kH; ++c) acc = fmaf(W2s[(7 * g + q) * kH + c], h[2][c], acc);
                os[q] = acc;
            }
            const float* O = a.offsets + ((int64_t)aid * a.k + g) * 3;
            float Ov[3] = {O[0], O[1], O[2]};
            write_gaussian(a, line * a.k + g, x, sc, Ov, oa, oc, os);
        }
    }
}

// ------------------------------------------------------------- compose
// G_t = [(i, j) : i visible ascending, j ascending, alpha_ij > 0]; each entry
// is the cache entry (line * k + j).
__global__ __launch_bounds__(NT) void k_compose_count(const int32_t* __restrict__ vslot, const float4* __restrict__ L0,
                                                      int k, Counters* cnt, uint32_t* __restrict__ count) {
    int32_t nv = cnt->n_visible;
    for (int64_t i = gtid(); i < nv; i += gstride()) {
        if (vslot[i] < 0) {  // anchor left without a line (capacity overflow)
            count[i] = 0u;
            continue;
        }
        int64_t base = (int64_t)vslot[i] * k;
        uint32_t c = 0;
        for (int j = 0; j < k; ++j) c += L0[base + j].w > 0.f ? 1u : 0u;
        count[i] = c;
    }
}

__global__ __launch_bounds__(NT) void k_compose_write(const int32_t* __restrict__ vslot, const float4* __restrict__ L0,
                                                      int k, Counters* cnt, const uint32_t* __restrict__ off,
                                                      int32_t* __restrict__ G) {
    int32_t nv = cnt->n_visible;
    for (int64_t i = gtid(); i < nv; i += gstride()) {
        if (vslot[i] < 0) continue;
        int64_t base = (int64_t)vslot[i] * k;
        uint32_t o = off[i];
        for (int j = 0; j < k; ++j)
            if (L0[base + j].w > 0.f) G[o++] = (int32_t)(base + j);
    }
}

inline dim3 grid_for(int64_t n) {
    int64_t b = (n + NT - 1) / NT;
    if (b < 1) b = 1;
    if (b > kGridBlocks) b = kGridBlocks;
    return dim3((unsigned)b);
}

}  // namespace

WeightLayout weight_layout(int k) {
    WeightLayout L;
    const int c[3] = {1, 3, 7};
    int off = 0, soff = 0;
    for (int h = 0; h < 3; ++h) {
        L.rows1[h] = kH;
        L.rows2[h] = c[h] * k;
        L.W1[h] = off; off += kH * (kF + 3);
        L.b1[h] = off; off += kH;
        L.W2[h] = off; off += c[h] * k * kH;
        L.b2[h] = off; off += c[h] * k;
        L.scale_W1[h] = soff; soff += kH;
        L.scale_W2[h] = soff; soff += c[h] * k;
    }
    // pad so that bf16 / fp8 copies stay 16-byte aligned per array
    L.total = (off + 15) / 16 * 16;
    L.scale_total = soff;
    return L;
}

#define GSC_TRY(x)                              \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

hipError_t derive_frame(const DeriveArgs& a, hipStream_t st) {
    const Scene& sc = *a.sc;
    View& v = *a.v;
    const int64_t n = sc.n;
    const int32_t t = (int32_t)v.t;
    Counters* cnt = v.cnt;
    hipLaunchKernelGGL(k_frame_begin, dim3(1), dim3(1), 0, st, cnt);
    hipLaunchKernelGGL(k_store_pu, dim3(1), dim3(64), 0, st, v.pu_hist, t, a.cam);
    // anchor indexing and filtering -> X_t ascending
    hipLaunchKernelGGL(k_select_flags, grid_for(n), dim3(NT), 0, st, sc.posr, sc.level, n, a.cam, v.tmp_a);
    GSC_TRY(scan_u32(v.tmp_a, v.tmp_b, nullptr, n, &cnt->n_visible, v.block_sums, st));
    hipLaunchKernelGGL(k_compact_ids, grid_for(n), dim3(NT), 0, st, v.tmp_a, v.tmp_b, n, nullptr, v.visible);

    const bool reuse = (a.flags & GSC_FLAG_REUSE) != 0;
    if (!reuse) {
        hipLaunchKernelGGL(k_nocache, grid_for(n), dim3(NT), 0, st, v.misses, v.vslot, cnt);
    } else {
        const int64_t C = v.C;
        hipLaunchKernelGGL(k_cache_invalidate, grid_for(C), dim3(NT), 0, st, v.line_anchor, v.line_tau, v.slot_of, C,
                           t, cnt);
        LookupArgs la;
        la.visible = v.visible; la.slot_of = v.slot_of; la.line_last = v.line_last; la.line_tau = v.line_tau;
        la.miss_flag = v.tmp_a; la.t = t; la.reuse = 1;
        la.predictor = (a.flags & GSC_FLAG_PREDICTOR) ? 1 : 0;
        la.thr = a.pred_thr; la.posr = sc.posr; la.level = sc.level; la.scale = sc.scale; la.pu_hist = v.pu_hist;
        la.lmax = sc.l_max; la.dmax = a.d_max; la.cam = a.cam; la.pred_wbf = a.pred_wbf; la.pred_w32 = a.pred_w;
        la.cand_feat = a.collect ? v.cand_feat : nullptr; la.cand_id = v.cand_id; la.cnt = cnt;
        hipLaunchKernelGGL(k_cache_lookup, grid_for(n), dim3(NT), 0, st, la);
        // misses, ascending visible position (= ascending anchor id)
        GSC_TRY(scan_u32(v.tmp_a, v.tmp_b, &cnt->n_visible, 0, &cnt->n_miss, v.block_sums, st));
        hipLaunchKernelGGL(k_compact_ids, grid_for(n), dim3(NT), 0, st, v.tmp_a, v.tmp_b, 0, &cnt->n_visible,
                           v.misses);
        // misses that need a line, and their ranks
        uint32_t* need = v.tmp_a;
        uint32_t* need_rank = v.tmp_b;
        hipLaunchKernelGGL(k_need_flags, grid_for(n), dim3(NT), 0, st, v.misses, v.visible, v.slot_of, cnt, need);
        GSC_TRY(scan_u32(need, need_rank, &cnt->n_miss, 0, &cnt->n_need, v.block_sums, st));
        // free lines, ascending
        uint32_t* fflag = reinterpret_cast<uint32_t*>(v.tmp_c);
        uint32_t* fpos = reinterpret_cast<uint32_t*>(v.tmp_d);
        hipLaunchKernelGGL(k_free_flags, grid_for(C), dim3(NT), 0, st, v.line_anchor, C, fflag);
        GSC_TRY(scan_u32(fflag, fpos, nullptr, C, &cnt->n_free, v.block_sums, st));
        hipLaunchKernelGGL(k_compact_ids, grid_for(C), dim3(NT), 0, st, fflag, fpos, C, nullptr, v.free_list);
        // eviction of outdated lines when free lines are short
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, v.evict_hist, 64);
        hipLaunchKernelGGL(k_evict_hist, grid_for(C), dim3(NT), 0, st, v.line_anchor, v.line_last, C, t, a.d_max,
                           cnt, v.evict_hist);
        hipLaunchKernelGGL(k_evict_plan, dim3(1), dim3(1), 0, st, v.evict_hist, t, a.d_max, cnt, v.evict_scan_n, n);
        hipLaunchKernelGGL(k_evict_thr_flags, grid_for(n), dim3(NT), 0, st, v.slot_of, v.line_last, v.evict_scan_n,
                           cnt, fflag);
        GSC_TRY(scan_u32(fflag, fpos, v.evict_scan_n, 0, nullptr, v.block_sums, st));
        hipLaunchKernelGGL(k_evict_apply, grid_for(C), dim3(NT), 0, st, v.line_anchor, v.line_last, v.slot_of, fpos,
                           C, t, cnt);
        // free list again if anything was evicted (count 0 otherwise)
        hipLaunchKernelGGL(k_evict_freescan_n, dim3(1), dim3(1), 0, st, cnt, v.evict_scan_n, C);
        hipLaunchKernelGGL(k_free_flags_n, grid_for(C), dim3(NT), 0, st, v.line_anchor, v.evict_scan_n, fflag);
        GSC_TRY(scan_u32(fflag, fpos, v.evict_scan_n, 0, nullptr, v.block_sums, st));
        hipLaunchKernelGGL(k_compact_ids, grid_for(C), dim3(NT), 0, st, fflag, fpos, 0, v.evict_scan_n, v.free_list);
        hipLaunchKernelGGL(k_assign, grid_for(n), dim3(NT), 0, st, v.misses, v.visible, v.slot_of, v.line_anchor,
                           v.line_tau, v.line_last, need, need_rank, v.free_list, t, C, cnt);
        hipLaunchKernelGGL(k_vslot, grid_for(n), dim3(NT), 0, st, v.visible, v.slot_of, v.vslot, cnt);
    }
    // decode the misses
    if (a.precision == GSC_PREC_F32) {
        DeriveK dk;
        dk.posr = sc.posr; dk.feat = sc.feat; dk.scale = sc.scale; dk.offsets = sc.offsets; dk.w = sc.w32;
        dk.L = weight_layout(sc.k); dk.k = sc.k; dk.visible = v.visible; dk.misses = v.misses; dk.vslot = v.vslot;
        dk.L0 = v.L0; dk.L1 = v.L1; dk.L2 = v.L2; dk.L3 = v.L3; dk.cam = a.cam; dk.cnt = cnt;
        hipLaunchKernelGGL(k_derive_f32, grid_for(n), dim3(NT), 0, st, dk);
    } else {
        MfmaDeriveArgs m;
        m.posr = sc.posr; m.feat = sc.feat; m.scale = sc.scale; m.offsets = sc.offsets; m.w32 = sc.w32;
        m.wbf16 = sc.wbf16; m.wfp8 = sc.wfp8; m.wfp8_scale = sc.wfp8_scale; m.L = weight_layout(sc.k); m.k = sc.k;
        m.visible = v.visible; m.misses = v.misses; m.vslot = v.vslot; m.L0 = v.L0; m.L1 = v.L1; m.L2 = v.L2;
        m.L3 = v.L3; m.cam_pos[0] = a.cam.pos[0]; m.cam_pos[1] = a.cam.pos[1]; m.cam_pos[2] = a.cam.pos[2];
        m.n_miss = &cnt->n_miss; m.fp8 = a.precision == GSC_PREC_FP8;
        GSC_TRY(derive_mfma(m, n, st));
    }
    hipLaunchKernelGGL(k_depth_update, dim3(1), dim3(1), 0, st, cnt, a.d_max, a.guide);
    // compose the render buffer
    hipLaunchKernelGGL(k_compose_count, grid_for(n), dim3(NT), 0, st, v.vslot, v.L0, sc.k, cnt, v.tmp_a);
    GSC_TRY(scan_u32(v.tmp_a, v.tmp_b, &cnt->n_visible, 0, &cnt->n_gauss, v.block_sums, st));
    hipLaunchKernelGGL(k_compose_write, grid_for(n), dim3(NT), 0, st, v.vslot, v.L0, sc.k, cnt, v.tmp_b, v.G);
    return hipGetLastError();
}

}  // namespace gsc
