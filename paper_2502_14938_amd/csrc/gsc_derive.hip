// Derive stage of one frame of one viewer (Section 4, Alg. 1):
//   anchor indexing + filtering  -> k_select_flags + compaction (X_t, ascending)
//   cache scheduling             -> k_cache_* (invalidate at the reuse depth,
//                                   hit/miss, learned staleness, slot
//                                   allocation, eviction of outdated lines)
//   decode new anchors           -> derive_mfma (eq. 3, eq. 2; matrix cores)
//   configure the cache depth    -> depth_update (eq. 4, linear guide), in k_compose_reduce
//   update the render buffer     -> k_compose_* (opacity mask, Section 6)
// Every count stays on the device (Counters); the host only enqueues.
#include <cmath>

#include "gsc_blockscan.h"
#include "gsc_common.h"
#include "gsc_derive_mfma.h"
#include "gsc_pred_bf16.h"

namespace gsc {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// Per-frame counters reset, and the unified camera centre of frame t kept
// for the reuse features of later frames (run by the first block of the
// selection kernel).
__device__ __forceinline__ void frame_begin(Counters* cnt, float* pu_hist, int32_t t, const DeriveCam& cam) {
    if (threadIdx.x == 0) {
        cnt->n_cand = 0;
        cnt->overflow = 0;
        cnt->n_evict = 0;
        cnt->evict_short = 0;
    }
    if (threadIdx.x < 3) pu_hist[4 * (t & 63) + threadIdx.x] = cam.pos[threadIdx.x];
}

// ------------------------------------------------------------- selection
// Keep anchor a iff (level 0 or |x - p_u| <= d_ref 2^-level, or < 2 d_ref
// 2^-level with the fractional level transition) and its bounding sphere is
// not wholly outside any unified-frustum plane (4 sides + near).
// Direct-mapped cache (line_anchor non-null: line a can only hold anchor a):
// the invalidation of Alg. 1 is done here too, anchor a's line dropped when
// its age exceeds the current depth (the depth is the previous frame's
// update; starting the frame leaves it alone).
__global__ __launch_bounds__(NT) void k_select_flags(const float4* __restrict__ posr, const uint8_t* __restrict__ level,
                                                     int64_t n, DeriveCam cam, uint32_t* __restrict__ flags,
                                                     Counters* cnt, float* __restrict__ pu_hist, int32_t t,
                                                     int32_t* __restrict__ line_anchor, const int32_t* __restrict__ line_tau,
                                                     int32_t* __restrict__ slot_of) {
    if (blockIdx.x == 0) frame_begin(cnt, pu_hist, t, cam);
    const int32_t depth = cnt->depth;
    for (int64_t a = gtid(); a < n; a += gstride()) {
        if (line_anchor && line_anchor[a] >= 0 && t - line_tau[a] > depth) {
            slot_of[a] = -1;
            line_anchor[a] = -1;
        }
        float4 p = posr[a];
        int l = level[a];
        bool keep = true;
        if (l != 0) {
            float vx = p.x - cam.pos[0], vy = p.y - cam.pos[1], vz = p.z - cam.pos[2];
            float lim = ldexpf(cam.d_ref, -l);
            float d2 = vx * vx + vy * vy + vz * vz;
            // with the fractional transition a level stays until its weight
            // clamp(2 - dist / d_l, 0, 1) reaches 0 (the weight is applied
            // by the rasteriser's preprocess)
            keep = cam.fade ? d2 < 4.f * lim * lim : d2 <= lim * lim;
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
    // direct-mapped cache: a miss takes line aid here, and every visible
    // anchor's render-buffer line is its own id
    int32_t direct;
    int32_t* slot_of_w;
    int32_t* line_anchor;
    int32_t* line_tau_w;
    int32_t* vslot;
};

// Direct-mapped lines, used when there is a line for every anchor: anchor a
// owns line a.  Free lines can then never run short, so there is no free
// list and no eviction, and the hit/miss decisions are the same as with any
// other choice of free line.  Misses (re)take their line at frame t (here,
// in the lookup); every visible anchor's buffer position points at its own
// line.
//
// Hit iff the anchor still owns a line (after invalidation every owned line
// has 1 <= t - tau <= d_t), reuse is on and the predictor does not flag it.
// Every visible owned line is stamped last_used = t.  The loop is uniform
// per wave: the predictor runs on the whole wave (matrix cores) whenever one
// of its lanes has a candidate.
__global__ __launch_bounds__(NT) void k_cache_lookup(LookupArgs a) {
    __shared__ uint32_t s_h[NT / 64][kPredLdsWave];
    const int32_t nv = a.cnt->n_visible;
    const int lane = threadIdx.x & 63;
    for (int64_t w0 = gtid() - lane; w0 < nv; w0 += gstride()) {
        const int64_t i = w0 + lane;
        const bool valid = i < nv;
        bool hit = false;
        float f[kPredIn] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int32_t aid = 0, s = -1;
        if (valid) {
            aid = a.visible[i];
            s = a.slot_of[aid];
            hit = s >= 0 && a.reuse;
            if (s >= 0) a.line_last[s] = a.t;
            if (hit && (a.predictor || a.cand_feat)) {
                const int32_t tau = a.line_tau[s];
                reuse_features(a.posr[aid], a.level[aid], a.lmax, a.scale + 6 * (int64_t)aid, a.cam.pos,
                               a.pu_hist + 4 * (tau & 63), a.t - tau, a.dmax, a.cam.fx, f);
                if (a.cand_feat) {
                    const int32_t c = atomicAdd(&a.cnt->n_cand, 1);
                    for (int q = 0; q < kPredIn; ++q) a.cand_feat[(int64_t)c * kPredIn + q] = f[q];
                    a.cand_id[c] = aid;
                }
            }
        }
        if (a.predictor && __any(hit)) {
            const float p = pred_prob_bf16_wave(a.pred_wbf, a.pred_w32, f, s_h[threadIdx.x >> 6]);
            if (hit && p > a.thr) hit = false;
        }
        if (valid) {
            a.miss_flag[i] = hit ? 0u : 1u;
            if (a.direct) {
                a.vslot[i] = aid;
                if (!hit) {  // derived this frame into line aid
                    if (s < 0) {
                        a.slot_of_w[aid] = aid;
                        a.line_anchor[aid] = aid;
                        a.line_last[aid] = a.t;
                    }
                    a.line_tau_w[aid] = a.t;
                }
            }
        }
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
__global__ __launch_bounds__(NT) void k_nocache(const int32_t* __restrict__ visible, int32_t* __restrict__ misses,
                                                int32_t* __restrict__ vslot, int32_t* __restrict__ line_anchor,
                                                Counters* cnt) {
    int32_t nv = cnt->n_visible;
    if (gtid() == 0) cnt->n_miss = nv;
    for (int64_t i = gtid(); i < nv; i += gstride()) {
        misses[i] = (int32_t)i;
        vslot[i] = (int32_t)i;
        line_anchor[i] = visible[i];
    }
}

// Eq. 4 with the linear guiding function on the update (miss) rate.
__device__ __forceinline__ void depth_update(Counters* cnt, int32_t dmax, int32_t guide) {
    int32_t nx = cnt->n_visible, nm = cnt->n_miss;
    cnt->depth_used = cnt->depth;
    if (guide == GSC_GUIDE_FIXED) {
        cnt->depth = dmax;
        return;
    }
    if (nx <= 0) return;
    int64_t d;
    if (guide == GSC_GUIDE_EXP) {
        const int64_t q = (8ll * nm) / nx;  // eighths of update rate
        d = q >= 31 ? 0 : ((int64_t)dmax >> q);
    } else if (guide == GSC_GUIDE_STAGED) {
        d = 8ll * nm < nx ? dmax : (8ll * nm < 3ll * nx ? dmax / 2 : 1);
    } else {  // linear: round_half_up(d_max (1 - r))
        d = (2ll * dmax * (nx - nm) + nx) / (2ll * nx);
    }
    cnt->depth = (int32_t)(d < 1 ? 1 : (d > dmax ? dmax : d));
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



// ------------------------------------------------------------- compose
// G_t = [(i, j) : i visible ascending, j ascending, alpha_ij > 0]; each entry
// is the cache entry (line * k + j).
static_assert(NT == blockscan::kThreads, "the fused compose scan uses the block-scan shape");

// Composition of the render buffer as one fused scan: visible anchor i
// contributes the Gaussians of its line whose opacity is positive (the
// line's mask, set by the derivation; none for an anchor left without a line
// at a capacity overflow), written to G in visible order at the exclusive
// prefix of the contributions.  The reduce pass sums each block's chunk and
// runs the depth update (eq. 4) from this frame's counts; the down-sweep
// writes the ids.
__device__ __forceinline__ uint32_t compose_mask(const int32_t* __restrict__ vslot,
                                                 const uint16_t* __restrict__ line_mask, int64_t i, int32_t& slot) {
    slot = vslot[i];
    return slot < 0 ? 0u : (uint32_t)line_mask[slot];
}

__global__ __launch_bounds__(NT) void k_compose_reduce(const int32_t* __restrict__ vslot,
                                                       const uint16_t* __restrict__ line_mask, Counters* cnt,
                                                       int32_t dmax, int32_t guide, uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t wsum[NT / 64];
    if (gtid() == 0) depth_update(cnt, dmax, guide);  // eq. 4, from this frame's counts
    int64_t b0, b1;
    blockscan::chunk_of(cnt->n_visible, blockscan::kTile, b0, b1);
    uint32_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += NT) {
        int32_t slot;
        s += (uint32_t)__popc(compose_mask(vslot, line_mask, i, slot));
    }
    const uint32_t t = blockscan::block_sum(s, wsum);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = t;
}

__global__ __launch_bounds__(NT) void k_compose_scatter(const int32_t* __restrict__ vslot,
                                                        const uint16_t* __restrict__ line_mask, int k, Counters* cnt,
                                                        const uint32_t* __restrict__ block_sums, int32_t* __restrict__ G) {
    __shared__ uint32_t wsum[NT / 64];
    uint32_t carry = blockscan::block_carry(block_sums, wsum, &cnt->n_gauss);
    int64_t b0, b1;
    blockscan::chunk_of(cnt->n_visible, blockscan::kTile, b0, b1);
    for (int64_t base = b0; base < b1; base += blockscan::kTile) {
        uint32_t mk[4], s = 0;
        int32_t slot[4];
        const int64_t i0 = base + threadIdx.x * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            mk[r] = 0u;
            slot[r] = -1;
            if (i0 + r < b1) mk[r] = compose_mask(vslot, line_mask, i0 + r, slot[r]);
            s += (uint32_t)__popc(mk[r]);
        }
        uint32_t tot;
        uint32_t o = carry + blockscan::block_excl_scan(s, wsum, tot);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gb = (int64_t)slot[r] * k;
            uint32_t m = mk[r];
            while (m) {
                const int j = __ffs(m) - 1;
                m &= m - 1u;
                G[o++] = (int32_t)(gb + j);
            }
        }
        carry += tot;
    }
}

}  // namespace

#define GSC_TRY(x)                              \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

hipError_t derive_frame(const DeriveArgs& a, hipStream_t st, Marks* mk) {
    const Scene& sc = *a.sc;
    View& v = *a.v;
    const int64_t n = sc.n;
    const int32_t t = (int32_t)v.t;
    Counters* cnt = v.cnt;
    mark(mk, 0, st);
    // anchor indexing and filtering -> X_t ascending (the first block also
    // starts the frame's counters)
    const bool reuse = (a.flags & GSC_FLAG_REUSE) != 0;
    const bool direct = reuse && v.C >= n;  // line a holds anchor a or nothing
    hipLaunchKernelGGL(k_select_flags, grid_fit(k_select_flags, n), dim3(NT), 0, st, sc.posr, sc.level, n, a.cam, v.tmp_a,
                       cnt, v.pu_hist, t, direct ? v.line_anchor : nullptr, v.line_tau, v.slot_of);
    GSC_TRY(compact_u32(v.tmp_a, nullptr, n, &cnt->n_visible, v.visible, v.block_sums, st));

    if (!reuse) {
        hipLaunchKernelGGL(k_nocache, grid_fit(k_nocache, n), dim3(NT), 0, st, v.visible, v.misses, v.vslot,
                           v.line_anchor, cnt);
    } else {
        const int64_t C = v.C;
        if (!direct)  // (direct: done in k_select_flags)
            hipLaunchKernelGGL(k_cache_invalidate, grid_fit(k_cache_invalidate, C), dim3(NT), 0, st, v.line_anchor, v.line_tau,
                               v.slot_of, C, t, cnt);
        LookupArgs la;
        la.visible = v.visible; la.slot_of = v.slot_of; la.line_last = v.line_last; la.line_tau = v.line_tau;
        la.miss_flag = v.tmp_a; la.t = t; la.reuse = 1;
        la.predictor = (a.flags & GSC_FLAG_PREDICTOR) ? 1 : 0;
        la.thr = a.pred_thr; la.posr = sc.posr; la.level = sc.level; la.scale = sc.scale; la.pu_hist = v.pu_hist;
        la.lmax = sc.l_max; la.dmax = a.d_max; la.cam = a.cam; la.pred_wbf = a.pred_wbf; la.pred_w32 = a.pred_w;
        la.cand_feat = a.collect ? v.cand_feat : nullptr; la.cand_id = v.cand_id; la.cnt = cnt;
        la.direct = direct ? 1 : 0; la.slot_of_w = v.slot_of; la.line_anchor = v.line_anchor; la.line_tau_w = v.line_tau;
        la.vslot = v.vslot;
        hipLaunchKernelGGL(k_cache_lookup, grid_fit(k_cache_lookup, n), dim3(NT), 0, st, la);
        // misses, ascending visible position (= ascending anchor id)
        GSC_TRY(compact_u32(v.tmp_a, &cnt->n_visible, 0, &cnt->n_miss, v.misses, v.block_sums, st));
        if (!direct) {
            // misses that need a line, and their ranks
            uint32_t* need = v.tmp_a;
            uint32_t* need_rank = v.tmp_b;
            hipLaunchKernelGGL(k_need_flags, grid_fit(k_need_flags, n), dim3(NT), 0, st, v.misses, v.visible, v.slot_of, cnt, need);
            GSC_TRY(scan_u32(need, need_rank, &cnt->n_miss, 0, &cnt->n_need, v.block_sums, st));
            // free lines, ascending
            uint32_t* fflag = reinterpret_cast<uint32_t*>(v.tmp_c);
            uint32_t* fpos = reinterpret_cast<uint32_t*>(v.tmp_d);
            hipLaunchKernelGGL(k_free_flags, grid_fit(k_free_flags, C), dim3(NT), 0, st, v.line_anchor, C, fflag);
            GSC_TRY(scan_u32(fflag, fpos, nullptr, C, &cnt->n_free, v.block_sums, st));
            hipLaunchKernelGGL(k_compact_ids, grid_fit(k_compact_ids, C), dim3(NT), 0, st, fflag, fpos, C, nullptr, v.free_list);
            // eviction of outdated lines when free lines are short
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, v.evict_hist, 64);
            hipLaunchKernelGGL(k_evict_hist, grid_fit(k_evict_hist, C), dim3(NT), 0, st, v.line_anchor, v.line_last, C, t, a.d_max,
                               cnt, v.evict_hist);
            hipLaunchKernelGGL(k_evict_plan, dim3(1), dim3(1), 0, st, v.evict_hist, t, a.d_max, cnt, v.evict_scan_n, n);
            hipLaunchKernelGGL(k_evict_thr_flags, grid_fit(k_evict_thr_flags, n), dim3(NT), 0, st, v.slot_of, v.line_last, v.evict_scan_n,
                               cnt, fflag);
            GSC_TRY(scan_u32(fflag, fpos, v.evict_scan_n, 0, nullptr, v.block_sums, st));
            hipLaunchKernelGGL(k_evict_apply, grid_fit(k_evict_apply, C), dim3(NT), 0, st, v.line_anchor, v.line_last, v.slot_of, fpos,
                               C, t, cnt);
            // free list again if anything was evicted (count 0 otherwise)
            hipLaunchKernelGGL(k_evict_freescan_n, dim3(1), dim3(1), 0, st, cnt, v.evict_scan_n, C);
            hipLaunchKernelGGL(k_free_flags_n, grid_fit(k_free_flags_n, C), dim3(NT), 0, st, v.line_anchor, v.evict_scan_n, fflag);
            GSC_TRY(scan_u32(fflag, fpos, v.evict_scan_n, 0, nullptr, v.block_sums, st));
            hipLaunchKernelGGL(k_compact_ids, grid_fit(k_compact_ids, C), dim3(NT), 0, st, fflag, fpos, 0, v.evict_scan_n, v.free_list);
            hipLaunchKernelGGL(k_assign, grid_fit(k_assign, n), dim3(NT), 0, st, v.misses, v.visible, v.slot_of, v.line_anchor,
                               v.line_tau, v.line_last, need, need_rank, v.free_list, t, C, cnt);
            hipLaunchKernelGGL(k_vslot, grid_fit(k_vslot, n), dim3(NT), 0, st, v.visible, v.slot_of, v.vslot, cnt);
        }
    }
    // decode the misses on the matrix cores
    mark(mk, 1, st);
    {
        MfmaDeriveArgs m;
        m.posr = sc.posr; m.feat = sc.feat; m.scale = sc.scale; m.offsets = sc.offsets; m.k = sc.k;
        m.visible = v.visible; m.misses = v.misses; m.vslot = v.vslot; m.L0 = v.L0; m.L1 = v.L1; m.L2 = v.L2;
        m.L3 = v.L3; m.line_mask = v.line_mask; m.cam_pos[0] = a.cam.pos[0]; m.cam_pos[1] = a.cam.pos[1]; m.cam_pos[2] = a.cam.pos[2];
        m.inv_dist_unit = sc.dist_unit > 0.f ? 1.0f / sc.dist_unit : 0.f;
        m.n_miss = &cnt->n_miss; m.mode = a.precision;
        m.fr.l1_f32 = sc.fr_l1_f32; m.fr.l2_f32 = sc.fr_l2_f32; m.fr.l1_bf16 = sc.fr_l1_bf16;
        m.fr.l2_bf16 = sc.fr_l2_bf16; m.fr.l1_fp8 = sc.fr_l1_fp8; m.fr.l2_fp8 = sc.fr_l2_fp8;
        m.fr.b1 = sc.fr_b1; m.fr.b2 = sc.fr_b2; m.fr.s1 = sc.fr_s1; m.fr.s2 = sc.fr_s2;
        m.fr.n_at = sc.n_at; m.fr.n_ct = sc.n_ct; m.fr.n_vt = sc.n_vt;
        GSC_TRY(derive_mfma(m, n, st));
    }
    mark(mk, 2, st);
    // compose the render buffer
    hipLaunchKernelGGL(k_compose_reduce, dim3(kScanBlocks), dim3(NT), 0, st, v.vslot, v.line_mask, cnt, a.d_max, a.guide,
                       v.block_sums);
    hipLaunchKernelGGL(k_compose_scatter, dim3(kScanBlocks), dim3(NT), 0, st, v.vslot, v.line_mask, sc.k, cnt,
                       v.block_sums, v.G);
    mark(mk, 3, st);
    return hipGetLastError();
}

}  // namespace gsc
