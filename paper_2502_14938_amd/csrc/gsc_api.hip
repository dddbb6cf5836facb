// C ABI of libgscache (declared in include/gscache.h): context lifetime,
// scene loading, the stereo camera pair, and the frame entry points.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gsc_common.h"
#include "gsc_ctx.h"
#include "gsc_derive_mfma.h"

using namespace gsc;

namespace {

thread_local std::string g_err;

int fail(gsc_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_err = msg;
    return code;
}

int hip_fail(gsc_ctx* c, hipError_t e, const char* where) {
    return fail(c, GSC_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(c, x)                                   \
    do {                                                    \
        hipError_t e_ = (x);                                \
        if (e_ != hipSuccess) return hip_fail(c, e_, #x);   \
    } while (0)

}  // namespace

namespace gsc {

int global_fail(int code, const std::string& msg) { return fail(nullptr, code, msg); }

// --------------------------------------------------------- unified camera
// Binocular stereo de-redundancy (Section 4, eqs. 5-6), in double precision.

void unified_camera(const gsc_camera& l, const gsc_camera& r, gsc_camera& u) {
    double d[3], rt[3], dn[3];
    for (int i = 0; i < 3; ++i) d[i] = l.R[6 + i] + r.R[6 + i];
    double nd = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; ++i) d[i] /= nd;
    double bx = l.pos[0] - r.pos[0], by = l.pos[1] - r.pos[1], bz = l.pos[2] - r.pos[2];
    double setback = std::sqrt(bx * bx + by * by + bz * bz) / (2.0 * std::tan(0.5 * l.fovx));
    for (int i = 0; i < 3; ++i) rt[i] = l.R[i] + r.R[i];
    double pr = rt[0] * d[0] + rt[1] * d[1] + rt[2] * d[2];
    for (int i = 0; i < 3; ++i) rt[i] -= pr * d[i];
    double nr = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    for (int i = 0; i < 3; ++i) rt[i] /= nr;
    dn[0] = d[1] * rt[2] - d[2] * rt[1];
    dn[1] = d[2] * rt[0] - d[0] * rt[2];
    dn[2] = d[0] * rt[1] - d[1] * rt[0];
    u = l;
    for (int i = 0; i < 3; ++i) {
        u.R[i] = rt[i];
        u.R[3 + i] = dn[i];
        u.R[6 + i] = d[i];
        u.pos[i] = 0.5 * (l.pos[i] + r.pos[i]) - d[i] * setback;
    }
}

// Frustum planes of a camera in world space, inward: n.x + w >= -radius.
DeriveCam derive_cam(const gsc_camera& c, float d_ref, bool fade) {
    DeriveCam dc;
    dc.fade = fade ? 1 : 0;
    double tx = std::tan(0.5 * c.fovx), ty = std::tan(0.5 * c.fovy);
    double nx = std::sqrt(1.0 + tx * tx), ny = std::sqrt(1.0 + ty * ty);
    double cam_n[5][3] = {{0.0, 0.0, 1.0},
                          {1.0 / nx, 0.0, tx / nx},
                          {-1.0 / nx, 0.0, tx / nx},
                          {0.0, 1.0 / ny, ty / ny},
                          {0.0, -1.0 / ny, ty / ny}};
    for (int p = 0; p < 5; ++p) {
        double w[3];
        for (int j = 0; j < 3; ++j)
            w[j] = c.R[0 * 3 + j] * cam_n[p][0] + c.R[1 * 3 + j] * cam_n[p][1] + c.R[2 * 3 + j] * cam_n[p][2];
        double off = -(w[0] * c.pos[0] + w[1] * c.pos[1] + w[2] * c.pos[2]);
        if (p == 0) off -= c.znear;
        for (int j = 0; j < 3; ++j) dc.planes[p][j] = (float)w[j];
        dc.planes[p][3] = (float)off;
    }
    for (int i = 0; i < 3; ++i) dc.pos[i] = (float)c.pos[i];
    dc.d_ref = (float)d_ref;
    dc.fx = (float)(c.width / (2.0 * tx));
    return dc;
}

void seg_lod_fade(Seg& s, const Scene& sc, const gsc_camera& derive_camera) {
    s.level = sc.level;
    for (int i = 0; i < 3; ++i) s.upos[i] = (float)derive_camera.pos[i];  // as derive_cam rounds it
    s.d_ref = sc.d_ref;
}

bool valid_camera(const gsc_camera& c) {
    return c.width > 0 && c.height > 0 && c.fovx > 0 && c.fovx < M_PI && c.fovy > 0 && c.fovy < M_PI &&
           c.znear > 0 && std::isfinite(c.pos[0]) && std::isfinite(c.pos[1]) && std::isfinite(c.pos[2]);
}


hipError_t sync_all(gsc_ctx* c) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && c->blend_stream) e = hipStreamSynchronize(c->blend_stream);
    return e;
}

// Raster buffers of the last stereo frame.
Raster& stereo_raster(gsc_ctx* c) { return c->last_set ? c->raster2 : c->raster; }

void free_explicit(gsc_ctx* c) {
    if (c->xmem.empty()) return;
    (void)sync_all(c);
    c->xmem.release();
    c->xraster = Raster();
    c->xg = {};
    c->xg_cap = 0;
    c->xg_bytes = 0;
}

void free_labels(gsc_ctx* c) {
    if (c->lmem.empty()) return;
    (void)sync_all(c);
    c->lmem.release();
    c->lab_L0 = c->lab_L1 = c->lab_L2 = nullptr;
    c->lab_L3 = nullptr;
    c->lab_iota = nullptr;
    c->lab_y = nullptr;
    c->lab_entries = 0;
}

void free_all(gsc_ctx* c) {
    free_labels(c);
    if (c->mem.empty()) return;
    (void)sync_all(c);
    c->mem.release();
    c->scene = Scene();
    c->view[0] = View();
    c->view[1] = View();
    c->raster = Raster();
    c->raster2 = Raster();
    c->pipeline = false;
    c->blend_pending[0] = c->blend_pending[1] = false;
    c->last_set = 0;
    c->loaded = false;
}

// Buffers of one view (viewer): cache lines, slot map, per-frame lists and
// scratch.  A(p, count) allocates or only counts.
template <class Fn>
hipError_t view_layout(View& v, int64_t n, int64_t C, int k, Fn&& A) {
    const int64_t m = n > C ? n : C;
    hipError_t e;
#define A_(p, cnt) if ((e = A(p, cnt)) != hipSuccess) return e
    A_(v.slot_of, n); A_(v.line_anchor, C); A_(v.line_tau, C); A_(v.line_last, C);
    A_(v.L0, C * k); A_(v.L1, C * k); A_(v.L2, C * k); A_(v.L3, C * k); A_(v.line_mask, C);
    A_(v.pu_hist, 64 * 4); A_(v.visible, n); A_(v.vslot, n);
    A_(v.tmp_a, m); A_(v.tmp_b, m); A_(v.tmp_c, m); A_(v.tmp_d, m);
    A_(v.evict_hist, 64); A_(v.evict_scan_n, 1);
    A_(v.misses, n); A_(v.free_list, C); A_(v.G, C * k); A_(v.block_sums, kScanBlocks);
    A_(v.cand_feat, n * kPredIn); A_(v.cand_id, n); A_(v.cnt, 1);
#undef A_
    return hipSuccess;
}

struct ByteCounter {
    size_t bytes = 0;
    template <typename T>
    hipError_t operator()(T*&, int64_t count) {
        bytes += (size_t)(count > 0 ? count : 1) * sizeof(T);
        return hipSuccess;
    }
};

size_t view_bytes(int64_t n, int64_t C, int k) {
    View v;
    ByteCounter bc;
    (void)view_layout(v, n, C, k, bc);
    return bc.bytes;
}

size_t raster_bytes(int64_t max_entries, int64_t max_pairs, int64_t max_tiles, bool full_key) {
    Raster r;
    ByteCounter bc;
    (void)raster_layout(r, max_entries, max_pairs, max_tiles, full_key, bc);
    return bc.bytes;
}

hipError_t alloc_view(AllocSet& set, View& v, int64_t n, int64_t C, int k) {
    v.C = C;
    v.max_gauss = C * k;
    hipError_t e = view_layout(v, n, C, k, [&](auto*& p, int64_t cnt) { return dalloc(set, v.bytes, &p, cnt); });
    if (e != hipSuccess) return e;
    return halloc(set, &v.cnt_host, 1);
}

hipError_t alloc_raster(AllocSet& set, Raster& r, int64_t max_entries, int64_t max_pairs, int64_t max_tiles,
                        bool full_key) {
    r.max_entries = max_entries;
    r.max_pairs = max_pairs;
    r.max_tiles = max_tiles;
    r.srow_cap = max_entries;
    r.tall_cap = max_entries / 4 + 256;
    hipError_t e = raster_layout(r, max_entries, max_pairs, max_tiles, full_key,
                                 [&](auto*& p, int64_t cnt) { return dalloc(set, r.bytes, &p, cnt); });
    if (e != hipSuccess) return e;
    return halloc(set, &r.cnt_host, 1);
}

__global__ void k_reset_view(int32_t* slot_of, int64_t n, int32_t* line_anchor, int32_t* line_tau, int32_t* line_last,
                             int64_t C, Counters* cnt, int32_t dmax) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, st = (int64_t)gridDim.x * blockDim.x;
    for (int64_t a = i; a < n; a += st) slot_of[a] = -1;
    for (int64_t s = i; s < C; s += st) {
        line_anchor[s] = -1;
        line_tau[s] = 0;
        line_last[s] = 0;
    }
    if (i == 0) {
        Counters z = {};
        z.depth = dmax;
        z.depth_used = dmax;
        *cnt = z;
    }
}

hipError_t reset_view(View& v, int64_t n, int dmax, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_view, dim3(1024), dim3(256), 0, st, v.slot_of, n, v.line_anchor, v.line_tau,
                       v.line_last, v.C, v.cnt, dmax);
    v.t = 0;
    return hipGetLastError();
}

__global__ void k_pack_explicit(const float* __restrict__ mu, const float* __restrict__ cov,
                                const float* __restrict__ rgb, const float* __restrict__ alpha, int64_t n, float4* L0,
                                float4* L1, float4* L2, float* L3) {
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += st) {
        L0[i] = make_float4(mu[3 * i], mu[3 * i + 1], mu[3 * i + 2], alpha[i]);
        L1[i] = make_float4(cov[6 * i], cov[6 * i + 1], cov[6 * i + 2], cov[6 * i + 3]);
        L2[i] = make_float4(cov[6 * i + 4], cov[6 * i + 5], rgb[3 * i], rgb[3 * i + 1]);
        L3[i] = rgb[3 * i + 2];
    }
}

hipError_t pack_explicit(const gsc_gaussians& g, float4* L0, float4* L1, float4* L2, float* L3, hipStream_t st) {
    if (g.n <= 0) return hipSuccess;
    int64_t blocks = (g.n + 255) / 256;
    if (blocks > kGridBlocks) blocks = kGridBlocks;
    hipLaunchKernelGGL(k_pack_explicit, dim3((unsigned)blocks), dim3(256), 0, st, g.mu, g.cov, g.rgb, g.alpha, g.n,
                       L0, L1, L2, L3);
    return hipGetLastError();
}

hipError_t explicit_gaussians(gsc_ctx* c, const gsc_gaussians& g, int64_t ntiles) {
    int64_t need = g.n > 1 ? g.n : 1;
    if (c->xg_cap < need || c->xraster.max_tiles < ntiles) {
        free_explicit(c);
        int64_t cap = 1024;
        while (cap < need) cap <<= 1;
        int64_t pairs = c->cfg.max_pairs > 0 ? c->cfg.max_pairs : 64 * cap;
        if (pairs > (1ll << 31) - 1) pairs = (1ll << 31) - 1;
        int64_t tiles = ntiles > 1 ? ntiles : 1;
        hipError_t e = hipSuccess;
        if ((e = dalloc(c->xmem, c->xg_bytes, &c->xg.L0, cap)) == hipSuccess &&
            (e = dalloc(c->xmem, c->xg_bytes, &c->xg.L1, cap)) == hipSuccess &&
            (e = dalloc(c->xmem, c->xg_bytes, &c->xg.L2, cap)) == hipSuccess &&
            (e = dalloc(c->xmem, c->xg_bytes, &c->xg.L3, cap)) == hipSuccess)
            e = alloc_raster(c->xmem, c->xraster, cap, pairs, tiles, (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0);
        if (e != hipSuccess) {
            free_explicit(c);
            return e;
        }
        c->xg_cap = cap;
    }
    return pack_explicit(g, c->xg.L0, c->xg.L1, c->xg.L2, c->xg.L3, c->stream);
}

// Event set of the frame being issued (nullptr when timing is off).
Marks* frame_marks(gsc_ctx* c) {
    if (!c->timing) return nullptr;
    if (c->marks_used == c->marks.size()) {
        Marks m{};
        for (int i = 0; i <= kNumStages; ++i)
            // timing-only events: no system-scope fence (no cache writeback per mark)
            if (hipEventCreateWithFlags(&m.ev[i], hipEventDisableSystemFence) != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipEventDestroy(m.ev[j]);
                return nullptr;
            }
        c->marks.push_back(m);
    }
    Marks& m = c->marks[c->marks_used];
    // boundaries of the selected stages, and the frame's two ends
    uint32_t want = 1u | (1u << kNumStages);
    for (int i = 0; i < kNumStages; ++i)
        if (c->timing_mask >> i & 1u) want |= (1u << i) | (1u << (i + 1));
    m.want = want;
    return &m;
}

void free_marks(gsc_ctx* c) {
    for (Marks& m : c->marks)
        for (int i = 0; i <= kNumStages; ++i) (void)hipEventDestroy(m.ev[i]);
    c->marks.clear();
    c->marks_used = 0;
}

}  // namespace gsc

// ====================================================================== ABI

extern "C" {

int gsc_create(const gsc_config* cfg, void* stream, gsc_ctx** out) {
    if (!cfg || !out) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: null argument");
    *out = nullptr;
    if (cfg->k < 1 || cfg->k > kMaxK) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: k must be in [1, 16]");
    if (cfg->feat_dim != kF || cfg->hidden != kH)
        return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: feat_dim and hidden must be 32");
    if (cfg->d_max < 1 || cfg->d_max > 63) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: d_max must be in [1, 63]");
    if (cfg->precision < GSC_PREC_F32 || cfg->precision > GSC_PREC_FP8)
        return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: bad precision");
    if (cfg->guide < GSC_GUIDE_LINEAR || cfg->guide > GSC_GUIDE_STAGED)
        return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: bad guide");
    if (cfg->max_width < 1 || cfg->max_height < 1 || cfg->max_width > 16384 || cfg->max_height > 16384)
        return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: max image size out of range");
    if (cfg->cache_capacity < 0 || cfg->max_pairs < 0) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_create: negative size");
    gsc_ctx* c = new (std::nothrow) gsc_ctx();
    if (!c) return fail(nullptr, GSC_E_OOM, "gsc_create: out of host memory");
    c->cfg = *cfg;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, GSC_E_HIP, "gsc_create: no HIP device");
    }
    *out = c;
    return GSC_OK;
}

void gsc_destroy(gsc_ctx* c) {
    if (!c) return;
    (void)sync_all(c);
    gsc::free_marks(c);
    gsc::pred_free(c);
    gsc::free_explicit(c);
    gsc::free_all(c);
    for (int i = 0; i < 2; ++i) {
        if (c->front_done[i]) (void)hipEventDestroy(c->front_done[i]);
        if (c->blend_done[i]) (void)hipEventDestroy(c->blend_done[i]);
    }
    if (c->blend_stream) (void)hipStreamDestroy(c->blend_stream);
    delete c;
}

const char* gsc_last_error(const gsc_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int gsc_set_stream(gsc_ctx* c, void* stream) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_set_stream: null context");
    c->stream = (hipStream_t)stream;
    return GSC_OK;
}

int gsc_load_anchors(gsc_ctx* c, const gsc_anchors* an, const gsc_mlp* mlp) {
    if (!c || !an || !mlp) return fail(c, GSC_E_INVALID_ARG, "gsc_load_anchors: null argument");
    if (an->n < 1 || an->n > (1ll << 30)) return fail(c, GSC_E_INVALID_ARG, "gsc_load_anchors: n out of range");
    if (!an->pos || !an->level || !an->radius || !an->feat || !an->scale || !an->offsets)
        return fail(c, GSC_E_INVALID_ARG, "gsc_load_anchors: null array");
    for (int h = 0; h < 3; ++h)
        if (!mlp->W1[h] || !mlp->b1[h] || !mlp->W2[h] || !mlp->b2[h])
            return fail(c, GSC_E_INVALID_ARG, "gsc_load_anchors: null weight");
    if (!(an->d_ref > 0)) return fail(c, GSC_E_INVALID_ARG, "gsc_load_anchors: d_ref must be positive");
    if (!(an->dist_unit >= 0) || !std::isfinite(an->dist_unit))
        return fail(c, GSC_E_INVALID_ARG, "gsc_load_anchors: dist_unit must be 0 or positive");
    const int64_t n = an->n;
    const int k = c->cfg.k;
    free_all(c);
    HIP_OR_FAIL(c, hipSetDevice(c->device));

    // host copies of the inputs (device inputs are staged through the host)
    auto fetch = [&](const void* src, size_t bytes, std::vector<uint8_t>& buf) -> const void* {
        if (!an->is_device) return src;
        buf.resize(bytes);
        if (hipMemcpy(buf.data(), src, bytes, hipMemcpyDeviceToHost) != hipSuccess) return nullptr;
        return buf.data();
    };
    std::vector<uint8_t> bpos, blev, brad, bfeat, bscale, boff;
    const float* pos = (const float*)fetch(an->pos, n * 12, bpos);
    const uint8_t* lev = (const uint8_t*)fetch(an->level, n, blev);
    const float* rad = (const float*)fetch(an->radius, n * 4, brad);
    const float* feat = (const float*)fetch(an->feat, n * kF * 4, bfeat);
    const float* scl = (const float*)fetch(an->scale, n * 24, bscale);
    const float* off = (const float*)fetch(an->offsets, n * k * 12, boff);
    if (!pos || !lev || !rad || !feat || !scl || !off) return fail(c, GSC_E_HIP, "gsc_load_anchors: device read failed");

    Scene& sc = c->scene;
    sc.n = n;
    sc.k = k;
    sc.d_ref = (float)an->d_ref;
    sc.dist_unit = (float)an->dist_unit;
    int lmax = 0;
    for (int64_t a = 0; a < n; ++a) lmax = lev[a] > lmax ? lev[a] : lmax;
    sc.l_max = lmax;
    std::vector<float4> posr(n);
    for (int64_t a = 0; a < n; ++a) posr[a] = make_float4(pos[3 * a], pos[3 * a + 1], pos[3 * a + 2], rad[a]);

    const int nviews = (c->cfg.flags & GSC_FLAG_DEREDUNDANCY) ? 1 : 2;
    int64_t C = c->cfg.cache_capacity > 0 ? c->cfg.cache_capacity : n;
    // the no-cache schedule (reuse off, or per-eye views) derives visible anchor i into line i
    if ((!(c->cfg.flags & GSC_FLAG_REUSE) || nviews == 2) && C < n) C = n;
    const int64_t max_gauss = C * k;
    int64_t ntx = (c->cfg.max_width + kTile - 1) / kTile, nty = (c->cfg.max_height + kTile - 1) / kTile;
    int64_t max_entries = 2 * max_gauss;
    if (max_entries > (1ll << 31) - 1) max_entries = (1ll << 31) - 1;
    int64_t max_pairs = c->cfg.max_pairs > 0 ? c->cfg.max_pairs : 24 * max_entries;
    const int64_t pair_cap = (int64_t)1 << 28;
    if (c->cfg.max_pairs == 0 && max_pairs > pair_cap) max_pairs = pair_cap;
    if (max_pairs > (1ll << 31) - 1) max_pairs = (1ll << 31) - 1;

    size_t& b = sc.bytes;
    hipError_t e;
#define A_(p, cnt)                                                         \
    if ((e = dalloc(c->mem, b, &p, cnt)) != hipSuccess) {                       \
        free_all(c);                                                       \
        return fail(c, GSC_E_OOM, "gsc_load_anchors: device allocation"); \
    }
    A_(sc.posr, n); A_(sc.level, n); A_(sc.feat, n * kF); A_(sc.scale, n * 6); A_(sc.offsets, n * k * 3);
    HostFrags hf = pack_frags(*mlp, k, an->dist_unit > 0 ? kF + 4 : kF + 3);
    A_(sc.fr_l1_f32, hf.l1_f32.size()); A_(sc.fr_l2_f32, hf.l2_f32.size());
    A_(sc.fr_l1_bf16, hf.l1_bf16.size()); A_(sc.fr_l2_bf16, hf.l2_bf16.size());
    A_(sc.fr_l1_fp8, hf.l1_fp8.size()); A_(sc.fr_l2_fp8, hf.l2_fp8.size());
    A_(sc.fr_b1, hf.b1.size()); A_(sc.fr_b2, hf.b2.size()); A_(sc.fr_s1, hf.s1.size()); A_(sc.fr_s2, hf.s2.size());
    sc.n_at = hf.n_at; sc.n_ct = hf.n_ct; sc.n_vt = hf.n_vt;
#undef A_
    for (int vi = 0; vi < nviews; ++vi)
        if (alloc_view(c->mem, c->view[vi], n, C, k) != hipSuccess) {
            free_all(c);
            return fail(c, GSC_E_OOM, "gsc_load_anchors: view allocation");
        }
    c->rcap_entries = max_entries;
    c->rcap_pairs = max_pairs;
    c->rcap_tiles = 2 * ntx * nty;
    if (alloc_raster(c->mem, c->raster, max_entries, max_pairs, 2 * ntx * nty,
                     (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0) != hipSuccess) {
        free_all(c);
        return fail(c, GSC_E_OOM, "gsc_load_anchors: raster allocation");
    }
    hipStream_t st = c->stream;
    HIP_OR_FAIL(c, hipMemcpyAsync(sc.posr, posr.data(), n * sizeof(float4), hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(c, hipMemcpyAsync(sc.level, lev, n, hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(c, hipMemcpyAsync(sc.feat, feat, n * kF * 4, hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(c, hipMemcpyAsync(sc.scale, scl, n * 24, hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(c, hipMemcpyAsync(sc.offsets, off, n * k * 12, hipMemcpyHostToDevice, st));
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    HIP_OR_FAIL(c, up(sc.fr_l1_f32, hf.l1_f32.data(), hf.l1_f32.size() * 4));
    HIP_OR_FAIL(c, up(sc.fr_l2_f32, hf.l2_f32.data(), hf.l2_f32.size() * 4));
    HIP_OR_FAIL(c, up(sc.fr_l1_bf16, hf.l1_bf16.data(), hf.l1_bf16.size() * 2));
    HIP_OR_FAIL(c, up(sc.fr_l2_bf16, hf.l2_bf16.data(), hf.l2_bf16.size() * 2));
    HIP_OR_FAIL(c, up(sc.fr_l1_fp8, hf.l1_fp8.data(), hf.l1_fp8.size() * 2));
    HIP_OR_FAIL(c, up(sc.fr_l2_fp8, hf.l2_fp8.data(), hf.l2_fp8.size() * 2));
    HIP_OR_FAIL(c, up(sc.fr_b1, hf.b1.data(), hf.b1.size() * 4));
    HIP_OR_FAIL(c, up(sc.fr_b2, hf.b2.data(), hf.b2.size() * 4));
    HIP_OR_FAIL(c, up(sc.fr_s1, hf.s1.data(), hf.s1.size() * 4));
    HIP_OR_FAIL(c, up(sc.fr_s2, hf.s2.data(), hf.s2.size() * 4));
    for (int vi = 0; vi < nviews; ++vi) HIP_OR_FAIL(c, reset_view(c->view[vi], n, c->cfg.d_max, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(st));
    c->nviews = nviews;
    c->loaded = true;
    c->have_pair = false;
    c->derived = false;
    return GSC_OK;
}

int gsc_set_camera_pair(gsc_ctx* c, const gsc_camera* left, const gsc_camera* right, double t_arrival) {
    if (!c || !left || !right) return fail(c, GSC_E_INVALID_ARG, "gsc_set_camera_pair: null argument");
    if (!valid_camera(*left) || !valid_camera(*right))
        return fail(c, GSC_E_INVALID_ARG, "gsc_set_camera_pair: invalid camera");
    if (left->width != right->width || left->height != right->height || left->fovx != right->fovx ||
        left->fovy != right->fovy || left->znear != right->znear)
        return fail(c, GSC_E_INVALID_ARG, "gsc_set_camera_pair: eyes must share intrinsics");
    if (left->width > c->cfg.max_width || left->height > c->cfg.max_height)
        return fail(c, GSC_E_INVALID_ARG, "gsc_set_camera_pair: image larger than max_width x max_height");
    c->eye[0] = *left;
    c->eye[1] = *right;
    unified_camera(*left, *right, c->unified);
    c->t_arrival = t_arrival;
    c->have_pair = true;
    return GSC_OK;
}

int gsc_derive(gsc_ctx* c) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_derive: null context");
    if (!c->loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_derive: no scene loaded");
    if (!c->have_pair) return fail(c, GSC_E_NOT_LOADED, "gsc_derive: no camera pair set");
    if ((c->cfg.flags & GSC_FLAG_PREDICTOR) && !c->pred_loaded)
        return fail(c, GSC_E_NOT_LOADED, "gsc_derive: predictor flag set but no predictor loaded");
    for (int vi = 0; vi < c->nviews; ++vi) {
        DeriveArgs a;
        a.sc = &c->scene;
        a.v = &c->view[vi];
        const gsc_camera& cam = c->nviews == 1 ? c->unified : c->eye[vi];
        a.cam = derive_cam(cam, c->scene.d_ref, (c->cfg.flags & GSC_FLAG_LOD_FADE) != 0);
        a.precision = c->cfg.precision;
        a.flags = c->cfg.flags;
        if (c->nviews == 2) a.flags &= ~(GSC_FLAG_REUSE | GSC_FLAG_PREDICTOR);
        a.d_max = c->cfg.d_max;
        a.guide = c->cfg.guide;
        a.pred_thr = c->cfg.predictor_threshold;
        a.pred_w = c->pred_w;
        a.pred_wbf = c->pred_wbf;
        a.collect = c->collect_features;
        hipError_t e = derive_frame(a, c->stream, vi == 0 ? frame_marks(c) : nullptr);
        if (e != hipSuccess) return hip_fail(c, e, "gsc_derive");
        c->view[vi].t += 1;
    }
    c->frame = c->view[0].t - 1;
    c->derived = true;
    return GSC_OK;
}

int gsc_render_stereo(gsc_ctx* c, float* left_chw, float* right_chw, float* left_T, float* right_T) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_render_stereo: null context");
    if (!left_chw || !right_chw) return fail(c, GSC_E_INVALID_ARG, "gsc_render_stereo: null output");
    if (!c->derived) return fail(c, GSC_E_NOT_LOADED, "gsc_render_stereo: call gsc_derive first");
    SegTable tab;
    std::memset(&tab, 0, sizeof(tab));
    tab.n = 2;
    tab.paired = c->nviews == 1 ? 1 : 0;  // both eyes read one view's buffer
    int tiles = 0;
    float* outs[2] = {left_chw, right_chw};
    float* Ts[2] = {left_T, right_T};
    for (int e = 0; e < 2; ++e) {
        View& v = c->view[c->nviews == 1 ? 0 : e];
        Seg& s = tab.s[e];
        s.L0 = v.L0; s.L1 = v.L1; s.L2 = v.L2; s.L3 = v.L3; s.G = v.G; s.nG = &v.cnt->n_gauss; s.nG_host = 0;
        // direct-mapped cache (the schedule gives anchor a line a): the
        // line index is the anchor, no lookup needed
        const bool direct = (c->cfg.flags & GSC_FLAG_REUSE) && c->nviews == 1 && v.C >= c->scene.n;
        s.anchor_pos = c->scene.posr; s.line_anchor = direct ? nullptr : v.line_anchor; s.k = c->scene.k;
        seg_camera(s, c->eye[e]);
        if (c->cfg.flags & GSC_FLAG_LOD_FADE) seg_lod_fade(s, c->scene, c->nviews == 1 ? c->unified : c->eye[e]);
        s.tile_base = tiles;
        tiles += s.ntx * s.nty;
        s.out_rgb = outs[e];
        s.out_T = Ts[e];
        s.out_nc = nullptr;
    }
    tab.total_tiles = tiles;
    Marks* mk = frame_marks(c);
    // two frames in flight: this frame's set was last read by the blend two
    // frames back, which must finish before the preprocess rewrites it
    const int set = c->pipeline ? (int)(c->pipe_frames & 1) : 0;
    Raster& R = set ? c->raster2 : c->raster;
    hipError_t e = hipSuccess;
    if (c->pipeline && c->blend_pending[set]) e = hipStreamWaitEvent(c->stream, c->blend_done[set], 0);
    if (e == hipSuccess)
        e = raster_batch(tab, R, (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0, c->count_work, c->stream, mk,
                         c->pipeline ? c->blend_stream : nullptr, c->pipeline ? c->front_done[set] : nullptr);
    if (e == hipSuccess && c->pipeline) {
        e = hipEventRecord(c->blend_done[set], c->blend_stream);
        c->blend_pending[set] = e == hipSuccess;
        c->pipe_frames += 1;
    }
    if (e != hipSuccess) return hip_fail(c, e, "gsc_render_stereo");
    c->last_set = set;
    if (mk) c->marks_used += 1;
    c->last_count_work = c->count_work;
    c->last_tab = tab;
    c->rendered = true;
    c->explicit_render = false;
    return GSC_OK;
}

int gsc_render_gaussians(gsc_ctx* c, const gsc_gaussians* g, const gsc_camera* cam, float* out_chw, float* out_T,
                         int32_t* out_nc) {
    if (!c || !g || !cam || !out_chw) return fail(c, GSC_E_INVALID_ARG, "gsc_render_gaussians: null argument");
    if (g->n < 0 || (g->n > 0 && (!g->mu || !g->cov || !g->rgb || !g->alpha)))
        return fail(c, GSC_E_INVALID_ARG, "gsc_render_gaussians: bad Gaussian arrays");
    if (!valid_camera(*cam) || cam->width > c->cfg.max_width || cam->height > c->cfg.max_height)
        return fail(c, GSC_E_INVALID_ARG, "gsc_render_gaussians: invalid camera or image too large");
    if (g->n > (1ll << 30)) return fail(c, GSC_E_INVALID_ARG, "gsc_render_gaussians: too many Gaussians");
    int64_t ntiles = (int64_t)((cam->width + kTile - 1) / kTile) * ((cam->height + kTile - 1) / kTile);
    hipError_t e = explicit_gaussians(c, *g, ntiles);
    if (e != hipSuccess) return hip_fail(c, e, "gsc_render_gaussians");
    SegTable tab;
    std::memset(&tab, 0, sizeof(tab));
    tab.n = 1;
    Seg& s = tab.s[0];
    s.L0 = c->xg.L0; s.L1 = c->xg.L1; s.L2 = c->xg.L2; s.L3 = c->xg.L3; s.G = nullptr; s.nG = nullptr;
    s.anchor_pos = nullptr; s.line_anchor = nullptr; s.k = 1;
    s.nG_host = (int32_t)g->n;
    seg_camera(s, *cam);
    s.tile_base = 0;
    s.out_rgb = out_chw; s.out_T = out_T; s.out_nc = out_nc;
    tab.total_tiles = s.ntx * s.nty;
    e = raster_batch(tab, c->xraster, (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0, c->count_work || out_nc,
                     c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "gsc_render_gaussians");
    c->last_tab = tab;
    c->rendered = true;
    c->explicit_render = true;
    return GSC_OK;
}

int gsc_sync(gsc_ctx* c) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_sync: null context");
    HIP_OR_FAIL(c, sync_all(c));
    int of = 0;
    if (c->rendered) {
        Raster& R = c->explicit_render ? c->xraster : stereo_raster(c);
        HIP_OR_FAIL(c, hipMemcpy(R.cnt_host, R.cnt, sizeof(RasterCounters), hipMemcpyDeviceToHost));
        of |= (R.cnt_host->overflow & 7) ? 1 : 0;  // tile pairs, entries or tall-footprint rows
    }
    if (c->loaded && c->derived) {
        HIP_OR_FAIL(c, hipMemcpy(c->view[0].cnt_host, c->view[0].cnt, sizeof(Counters), hipMemcpyDeviceToHost));
        of |= c->view[0].cnt_host->overflow & 2;
    }
    if (of) return fail(c, GSC_E_CAPACITY, of & 1 ? "raster capacity exceeded (tile pairs, entries or tall-footprint rows)"
                                                  : "cache capacity exceeded");
    return GSC_OK;
}

}  // extern "C"

namespace gsc {
namespace {

// One image's depth-ordered tile lists, as the blend reads them: tile t's
// list is its super tile's sorted list filtered by the tile's mask bit.
// Fills the lists' concatenation in tile order (sorted pair values: entry |
// mask << kMaskShift) and start[t] (start[ntiles] = total).
hipError_t image_tile_lists(const SegTable& last, const Raster& R, int eye, std::vector<uint32_t>& vals,
                            std::vector<int64_t>& start) {
    SegTable tab = last;
    seg_supers(tab);
    const Seg& s = tab.s[eye];
    const int64_t nsup = (int64_t)s.nsx * s.nsy;
    std::vector<int32_t> rg(2 * (size_t)nsup);
    hipError_t e = hipMemcpy(rg.data(), R.ranges + 2 * (int64_t)s.sup_base, rg.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    // the image's super tiles are consecutive ids, so their lists form one
    // contiguous span of the sorted values
    int64_t lo = -1, hi = -1;
    for (int64_t q = 0; q < nsup; ++q)
        if (rg[2 * q + 1] > rg[2 * q]) {
            if (lo < 0) lo = rg[2 * q];
            hi = rg[2 * q + 1];
        }
    std::vector<uint32_t> sv(lo < 0 ? 0 : (size_t)(hi - lo));
    if (!sv.empty()) {
        e = hipMemcpy(sv.data(), R.pval[R.sorted_buf] + lo, sv.size() * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
    }
    vals.clear();
    start.assign((size_t)s.ntx * s.nty + 1, 0);
    for (int ty = 0; ty < s.nty; ++ty)
        for (int tx = 0; tx < s.ntx; ++tx) {
            const int64_t q = (int64_t)(ty >> kSupShift) * s.nsx + (tx >> kSupShift);
            const uint32_t bit = 1u << (kMaskShift + ((ty & 1) << 1) + (tx & 1));
            start[(size_t)ty * s.ntx + tx] = (int64_t)vals.size();
            for (int64_t i = rg[2 * q]; i < rg[2 * q + 1]; ++i)
                if (sv[(size_t)(i - lo)] & bit) vals.push_back(sv[(size_t)(i - lo)]);
        }
    start.back() = (int64_t)vals.size();
    return hipSuccess;
}

// Tile pairs of each image of the last stereo batch (the sum of its entries'
// tile counts), for the frame statistics.
hipError_t image_tile_pairs(const SegTable& tab, const Raster& R, const RasterCounters& r, int64_t out[2]) {
    out[0] = out[1] = 0;
    const int64_t ne = r.n_entries;
    if (ne <= 0) return hipSuccess;
    std::vector<uint32_t> nt((size_t)ne);
    hipError_t e = hipMemcpy(nt.data(), R.ntiles, nt.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    const int64_t stride = r.entry_stride > 1 ? r.entry_stride : 1;
    for (int sg = 0; sg < tab.n && sg < 2; ++sg) {
        int64_t b0, b1;
        if (stride > 1) {  // the pair (sg & ~1, sg | 1) interleaves its two images' entries
            const int q = sg & ~1;
            b0 = r.entry_base[q] + (sg & 1);
            b1 = r.entry_base[q + 2];
        } else {
            b0 = r.entry_base[sg];
            b1 = r.entry_base[sg + 1];
        }
        int64_t n = 0;
        for (int64_t i = b0; i < b1 && i < ne; i += stride) n += nt[(size_t)i];
        out[sg] = n;
    }
    return hipSuccess;
}

}  // namespace
}  // namespace gsc

extern "C" {

int gsc_get_stats(gsc_ctx* c, gsc_frame_stats* st) {
    if (!c || !st) return fail(c, GSC_E_INVALID_ARG, "gsc_get_stats: null argument");
    std::memset(st, 0, sizeof(*st));
    HIP_OR_FAIL(c, sync_all(c));
    if (!c->loaded) return GSC_OK;
    HIP_OR_FAIL(c, hipMemcpy(c->view[0].cnt_host, c->view[0].cnt, sizeof(Counters), hipMemcpyDeviceToHost));
    Raster& SR = stereo_raster(c);
    HIP_OR_FAIL(c, hipMemcpy(SR.cnt_host, SR.cnt, sizeof(RasterCounters), hipMemcpyDeviceToHost));
    const Counters& k = *c->view[0].cnt_host;
    const RasterCounters& r = *SR.cnt_host;
    st->frame = c->frame;
    st->n_visible = k.n_visible;
    st->n_miss = k.n_miss;
    st->n_gauss = k.n_gauss;
    if (c->rendered && !c->explicit_render && c->last_tab.total_tiles > 0) {
        // tile pairs per eye: the sum of its entries' tile counts
        int64_t np[2];
        HIP_OR_FAIL(c, image_tile_pairs(c->last_tab, SR, r, np));
        st->n_pairs[0] = np[0];
        st->n_pairs[1] = np[1];
    }
    st->n_evicted = k.n_evict;
    st->depth_used = k.depth_used;
    st->depth_next = k.depth;
    st->overflow = ((r.overflow & 7) ? 1 : 0) | (k.overflow & 2);
    st->n_tall = r.n_tall_e;
    size_t bytes = c->scene.bytes + c->view[0].bytes + c->view[1].bytes + c->raster.bytes + c->raster2.bytes + c->xg_bytes;
    st->device_bytes = (int64_t)bytes;
    if (c->rendered && !c->explicit_render && c->last_count_work && c->last_tab.total_tiles > 0) {
        std::vector<int32_t> te(2 * (size_t)c->last_tab.total_tiles);
        HIP_OR_FAIL(c, hipMemcpy(te.data(), SR.tile_eval, te.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int sg = 0; sg < c->last_tab.n && sg < 2; ++sg) {
            const Seg& g = c->last_tab.s[sg];
            int64_t ev = 0, co = 0;
            for (int t = 0; t < g.ntx * g.nty; ++t) {
                ev += te[2 * (size_t)(g.tile_base + t)];
                co += te[2 * (size_t)(g.tile_base + t) + 1];
            }
            st->n_eval[sg] = ev;
            st->n_contrib[sg] = co;
        }
    }
    return GSC_OK;
}

int gsc_count_work(gsc_ctx* c, int enable) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_count_work: null context");
    c->count_work = enable != 0;
    return GSC_OK;
}

int gsc_pipeline(gsc_ctx* c, int enable) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_pipeline: null context");
    HIP_OR_FAIL(c, sync_all(c));
    c->blend_pending[0] = c->blend_pending[1] = false;
    c->pipe_frames = 0;
    if (!enable) {
        c->pipeline = false;
        return GSC_OK;
    }
    if (!c->loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_pipeline: no scene loaded");
    if (!c->blend_stream) {
        HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->blend_stream, hipStreamNonBlocking));
        for (int i = 0; i < 2; ++i) {
            HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->front_done[i], hipEventDisableTiming));
            HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->blend_done[i], hipEventDisableTiming));
        }
    }
    if (c->raster2.bytes == 0 &&
        alloc_raster(c->mem, c->raster2, c->rcap_entries, c->rcap_pairs, c->rcap_tiles,
                     (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0) != hipSuccess) {
        c->raster2 = Raster();
        return fail(c, GSC_E_OOM, "gsc_pipeline: second raster buffer set");
    }
    c->pipeline = true;
    return GSC_OK;
}

int gsc_ssim(gsc_ctx* c, const float* a, const float* b, int32_t channels, int32_t height, int32_t width,
             double* out) {
    if (!c || !a || !b || !out) return fail(c, GSC_E_INVALID_ARG, "gsc_ssim: null argument");
    if (channels < 1 || channels > 65535 || height < 11 || width < 11 || height > 65536 || width > 65536)
        return fail(c, GSC_E_INVALID_ARG, "gsc_ssim: images of 1..65535 channels, at least 11 x 11 pixels");
    HIP_OR_FAIL(c, sync_all(c));  // the images may come from a frame still in flight
    const SsimWindow win = ssim_window();
    const int64_t nb = ssim_blocks(channels, height, width);
    double* buf = nullptr;  // [0]: total, [1..nb]: per-block sums
    HIP_OR_FAIL(c, hipMalloc((void**)&buf, (size_t)(nb + 1) * sizeof(double)));
    hipError_t e = ssim_launch(a, b, channels, height, width, win, buf + 1, buf, c->stream);
    double tot = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&tot, buf, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(c, e, "gsc_ssim");
    *out = tot / ((double)channels * (double)(height - 10) * (double)(width - 10));
    return GSC_OK;
}

int gsc_timing(gsc_ctx* c, int enable) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_timing: null context");
    HIP_OR_FAIL(c, sync_all(c));
    c->timing = enable != 0;
    c->marks_used = 0;
    for (Marks& m : c->marks) m.recorded = 0;
    return GSC_OK;
}

int gsc_timing_stages(gsc_ctx* c, uint32_t stage_mask) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_timing_stages: null context");
    c->timing_mask = stage_mask;
    return GSC_OK;
}

int gsc_timing_read(gsc_ctx* c, double* ms, int32_t n, double* frame_ms, int64_t frame_cap, int64_t* frames) {
    if (!c || !ms || n < 0 || frame_cap < 0 || (frame_cap > 0 && !frame_ms))
        return fail(c, GSC_E_INVALID_ARG, "gsc_timing_read: bad argument");
    HIP_OR_FAIL(c, sync_all(c));
    for (int32_t i = 0; i < n; ++i) ms[i] = 0.0;
    for (size_t f = 0; f < c->marks_used; ++f) {
        Marks& m = c->marks[f];
        for (int i = 0; i < kNumStages && i < n; ++i) {
            const uint32_t need = (1u << i) | (1u << (i + 1));
            if ((m.recorded & need) != need) continue;
            float t = 0.f;
            if (hipEventElapsedTime(&t, m.ev[i], m.ev[i + 1]) == hipSuccess) ms[i] += t;
        }
        if ((int64_t)f < frame_cap) {
            const uint32_t ends = 1u | (1u << kNumStages);
            float t = -1.f;
            if ((m.recorded & ends) == ends) (void)hipEventElapsedTime(&t, m.ev[0], m.ev[kNumStages]);
            frame_ms[f] = t;
        }
        m.recorded = 0;
    }
    if (frames) *frames = (int64_t)c->marks_used;
    c->marks_used = 0;
    return GSC_OK;
}

int gsc_reset_cache(gsc_ctx* c) {
    if (!c) return fail(nullptr, GSC_E_INVALID_ARG, "gsc_reset_cache: null context");
    if (!c->loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_reset_cache: no scene loaded");
    for (int vi = 0; vi < c->nviews; ++vi) HIP_OR_FAIL(c, reset_view(c->view[vi], c->scene.n, c->cfg.d_max, c->stream));
    c->derived = false;
    return GSC_OK;
}

int gsc_debug_copy(gsc_ctx* c, int what, int eye, void* dst, int64_t cap, int64_t* n) {
    if (!c || !n) return fail(c, GSC_E_INVALID_ARG, "gsc_debug_copy: null argument");
    if (!c->loaded && !c->explicit_render) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: nothing to copy");
    Raster& R = c->explicit_render ? c->xraster : stereo_raster(c);
    const bool view_item = what <= GSC_DBG_DERIVED || what == GSC_DBG_DEPTH;
    if (view_item && !c->loaded) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: no scene loaded");
    if (eye < 0 || eye > 1) return fail(c, GSC_E_INVALID_ARG, "gsc_debug_copy: eye must be 0 or 1");
    if (cap > 0 && !dst) return fail(c, GSC_E_INVALID_ARG, "gsc_debug_copy: null destination");
    HIP_OR_FAIL(c, sync_all(c));
    View& v = c->view[c->nviews == 1 ? 0 : eye];
    Counters kz = {};
    if (c->loaded) {
        HIP_OR_FAIL(c, hipMemcpy(v.cnt_host, v.cnt, sizeof(Counters), hipMemcpyDeviceToHost));
        kz = *v.cnt_host;
    }
    RasterCounters rz = {};
    if (c->rendered) {
        HIP_OR_FAIL(c, hipMemcpy(R.cnt_host, R.cnt, sizeof(RasterCounters), hipMemcpyDeviceToHost));
        rz = *R.cnt_host;
    }
    const Counters& k = kz;
    const RasterCounters& r = rz;
    int64_t count = 0;
    std::vector<uint8_t> tmp;
    switch (what) {
        case GSC_DBG_VISIBLE:
        case GSC_DBG_MISSES: {
            count = what == GSC_DBG_VISIBLE ? k.n_visible : k.n_miss;
            int64_t m = count < cap ? count : cap;
            if (m > 0) {
                if (what == GSC_DBG_VISIBLE) {
                    HIP_OR_FAIL(c, hipMemcpy(dst, v.visible, m * 4, hipMemcpyDeviceToHost));
                } else {
                    std::vector<int32_t> pos(m), vis(k.n_visible);
                    HIP_OR_FAIL(c, hipMemcpy(pos.data(), v.misses, m * 4, hipMemcpyDeviceToHost));
                    HIP_OR_FAIL(c, hipMemcpy(vis.data(), v.visible, (size_t)k.n_visible * 4, hipMemcpyDeviceToHost));
                    for (int64_t i = 0; i < m; ++i) ((int32_t*)dst)[i] = vis[pos[i]];
                }
            }
            break;
        }
        case GSC_DBG_GAUSS:
        case GSC_DBG_DERIVED: {
            count = k.n_gauss;
            int64_t m = count < cap ? count : cap;
            if (m <= 0) break;
            std::vector<int32_t> G(m), vslot(k.n_visible);
            HIP_OR_FAIL(c, hipMemcpy(G.data(), v.G, m * 4, hipMemcpyDeviceToHost));
            if (what == GSC_DBG_GAUSS) {
                HIP_OR_FAIL(c, hipMemcpy(vslot.data(), v.vslot, (size_t)k.n_visible * 4, hipMemcpyDeviceToHost));
                // cache entry (line * k + j) -> (visible position * k + j)
                std::vector<int64_t> pos_of_line;
                int64_t kk = c->scene.k;
                std::vector<int32_t> inv((size_t)v.C, -1);
                for (int64_t i = 0; i < k.n_visible; ++i)
                    if (vslot[i] >= 0) inv[vslot[i]] = (int32_t)i;
                for (int64_t i = 0; i < m; ++i) ((int32_t*)dst)[i] = (int32_t)(inv[G[i] / kk] * kk + G[i] % kk);
            } else {
                int64_t E = v.C * c->scene.k;
                std::vector<float4> l0(E), l1(E), l2(E);
                std::vector<float> l3(E);
                HIP_OR_FAIL(c, hipMemcpy(l0.data(), v.L0, E * 16, hipMemcpyDeviceToHost));
                HIP_OR_FAIL(c, hipMemcpy(l1.data(), v.L1, E * 16, hipMemcpyDeviceToHost));
                HIP_OR_FAIL(c, hipMemcpy(l2.data(), v.L2, E * 16, hipMemcpyDeviceToHost));
                HIP_OR_FAIL(c, hipMemcpy(l3.data(), v.L3, E * 4, hipMemcpyDeviceToHost));
                // positions are stored relative to the line's anchor
                std::vector<int32_t> la((size_t)v.C);
                std::vector<float4> ap((size_t)c->scene.n);
                HIP_OR_FAIL(c, hipMemcpy(la.data(), v.line_anchor, la.size() * 4, hipMemcpyDeviceToHost));
                HIP_OR_FAIL(c, hipMemcpy(ap.data(), c->scene.posr, ap.size() * 16, hipMemcpyDeviceToHost));
                float* o = (float*)dst;
                for (int64_t i = 0; i < m; ++i) {
                    int64_t e = G[i];
                    const float4 a = ap[(size_t)la[(size_t)(e / c->scene.k)]];
                    float row[13] = {(float)((double)a.x + l0[e].x), (float)((double)a.y + l0[e].y),
                                     (float)((double)a.z + l0[e].z), l1[e].x, l1[e].y, l1[e].z, l1[e].w,
                                     l2[e].x, l2[e].y, l2[e].z, l2[e].w, l3[e], l0[e].w};
                    std::memcpy(o + 13 * i, row, sizeof(row));
                }
            }
            break;
        }
        case GSC_DBG_PAIRS: {
            if (!c->rendered) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: nothing rendered");
            const SegTable& tab = c->last_tab;
            if (eye >= tab.n) return fail(c, GSC_E_INVALID_ARG, "gsc_debug_copy: no such eye");
            const Seg& s = tab.s[eye];
            std::vector<uint32_t> val;
            std::vector<int64_t> st0;
            HIP_OR_FAIL(c, image_tile_lists(tab, R, eye, val, st0));
            count = (int64_t)val.size();
            int64_t m = count < cap ? count : cap;
            if (m <= 0) break;
            if (R.order) {  // pair values are depth ranks: map them back to entries
                int32_t ne = r.n_entries;
                std::vector<uint32_t> ord(ne > 0 ? ne : 1);
                if (ne > 0) HIP_OR_FAIL(c, hipMemcpy(ord.data(), R.order, (size_t)ne * 4, hipMemcpyDeviceToHost));
                for (auto& v : val) {
                    const uint32_t x = v & kEntryMask;
                    v = x < (uint32_t)ne ? ord[x] : kEntryMask;
                }
            }
            int32_t* o = (int32_t*)dst;
            const uint32_t stride = r.entry_stride > 1 ? (uint32_t)r.entry_stride : 1u;
            int64_t i = 0;
            for (int64_t t = 0; t < (int64_t)s.ntx * s.nty && i < m; ++t)
                for (int64_t j = st0[(size_t)t]; j < st0[(size_t)t + 1] && i < m; ++j, ++i) {
                    o[2 * i] = (int32_t)t;
                    o[2 * i + 1] = (int32_t)(((val[(size_t)j] & kEntryMask) - (uint32_t)r.entry_base[eye]) / stride);
                }
            break;
        }
        case GSC_DBG_RANGES: {
            if (!c->rendered) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: nothing rendered");
            const SegTable& tab = c->last_tab;
            if (eye >= tab.n) return fail(c, GSC_E_INVALID_ARG, "gsc_debug_copy: no such eye");
            const Seg& s = tab.s[eye];
            count = (int64_t)s.ntx * s.nty;
            int64_t m = count < cap ? count : cap;
            if (m <= 0) break;
            std::vector<uint32_t> val;
            std::vector<int64_t> st0;
            HIP_OR_FAIL(c, image_tile_lists(tab, R, eye, val, st0));
            int32_t* o = (int32_t*)dst;
            for (int64_t t = 0; t < m; ++t) {
                const bool empty = st0[(size_t)t + 1] <= st0[(size_t)t];
                o[2 * t] = empty ? 0 : (int32_t)st0[(size_t)t];
                o[2 * t + 1] = empty ? 0 : (int32_t)st0[(size_t)t + 1];
            }
            break;
        }
        case GSC_DBG_PREPROC: {
            if (!c->rendered) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: nothing rendered");
            if (eye >= c->last_tab.n) return fail(c, GSC_E_INVALID_ARG, "gsc_debug_copy: no such eye");
            // the eye's entries: from entry_base[eye] with the layout's stride
            const int64_t stride = r.entry_stride > 1 ? r.entry_stride : 1;
            const int64_t b0 = r.entry_base[eye];
            if (stride > 1) {  // the pair (eye & ~1, eye | 1) holds 2 entries per Gaussian
                const int q = eye & ~1;
                count = (r.entry_base[q + 2] - r.entry_base[q]) / 2;
            } else {
                count = r.entry_base[eye + 1] - b0;
            }
            int64_t m = count < cap ? count : cap;
            if (m <= 0) break;
            const int64_t span = (m - 1) * stride + 1;
            std::vector<float4> rr(4 * span);
            std::vector<uint32_t> nt(span);
            HIP_OR_FAIL(c, hipMemcpy(rr.data(), R.rec + 4 * b0, span * 64, hipMemcpyDeviceToHost));
            HIP_OR_FAIL(c, hipMemcpy(nt.data(), R.ntiles + b0, span * 4, hipMemcpyDeviceToHost));
            float* o = (float*)dst;
            for (int64_t i = 0; i < m; ++i) {
                const float4& A = rr[4 * i * stride];
                const float4& B = rr[4 * i * stride + 1];
                float row[8] = {A.x, A.y, A.z, A.w, B.x, B.y, 0.f, (float)nt[i * stride]};
                std::memcpy(o + 8 * i, row, sizeof(row));
            }
            break;
        }
        case GSC_DBG_DEPTH: {
            count = 1;
            if (cap >= 1) ((int32_t*)dst)[0] = k.depth;
            break;
        }
        case GSC_DBG_SORT_KEYS: {
            if (!c->rendered) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: nothing rendered");
            int32_t ns = 0;
            HIP_OR_FAIL(c, hipMemcpy(&ns, R.n_sort, sizeof(int32_t), hipMemcpyDeviceToHost));
            count = ns;
            int64_t m = count < cap ? count : cap;
            if (m <= 0) break;
            if (R.pkey64[R.sorted_buf] && (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT)) {
                std::vector<uint64_t> k64(m);
                HIP_OR_FAIL(c, hipMemcpy(k64.data(), R.pkey64[R.sorted_buf], m * 8, hipMemcpyDeviceToHost));
                for (int64_t i = 0; i < m; ++i) ((uint32_t*)dst)[i] = (uint32_t)(k64[i] >> 32);
            } else if (R.key16) {
                std::vector<uint16_t> k16(m);
                HIP_OR_FAIL(c, hipMemcpy(k16.data(), R.pkey[R.sorted_buf], m * 2, hipMemcpyDeviceToHost));
                for (int64_t i = 0; i < m; ++i) ((uint32_t*)dst)[i] = k16[i];
            } else {
                HIP_OR_FAIL(c, hipMemcpy(dst, R.pkey[R.sorted_buf], m * 4, hipMemcpyDeviceToHost));
            }
            break;
        }
        case GSC_DBG_SORT_VALS: {
            if (!c->rendered) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: nothing rendered");
            int32_t ns = 0;
            HIP_OR_FAIL(c, hipMemcpy(&ns, R.n_sort, sizeof(int32_t), hipMemcpyDeviceToHost));
            count = ns;
            int64_t m = count < cap ? count : cap;
            if (m > 0) HIP_OR_FAIL(c, hipMemcpy(dst, R.pval[R.sorted_buf], m * 4, hipMemcpyDeviceToHost));
            break;
        }
        case GSC_DBG_RAW_RANGES: {
            if (!c->rendered) return fail(c, GSC_E_NOT_LOADED, "gsc_debug_copy: nothing rendered");
            SegTable tab = c->last_tab;
            seg_supers(tab);
            count = tab.total_sup;
            int64_t m = count < cap ? count : cap;
            if (m > 0) HIP_OR_FAIL(c, hipMemcpy(dst, R.ranges, 2 * m * 4, hipMemcpyDeviceToHost));
            break;
        }
        default:
            return fail(c, GSC_E_INVALID_ARG, "gsc_debug_copy: unknown item");
    }
    *n = count;
    return GSC_OK;
}

}  // extern "C"
