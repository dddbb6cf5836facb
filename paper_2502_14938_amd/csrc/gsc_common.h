// Internal declarations shared by the libgscache translation units.
// Not part of the public ABI (include/gscache.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gscache.h"

namespace gsc {

constexpr int kTile = 16;             // 16x16 pixel tiles
// Binning unit of the sort: a super tile of 2x2 tiles (32x32 pixels).  A
// (super tile, entry) pair carries in its value the entry id and a 4-bit
// mask of the tiles of the super tile the footprint covers (bit
// 2 (ty & 1) + (tx & 1)); each tile's depth-ordered list is its super
// tile's list filtered by its bit.
constexpr int kSupShift = 1;          // log2 tiles per super-tile side
constexpr int kMaskShift = 28;        // value = entry | mask << kMaskShift
constexpr uint32_t kEntryMask = (1u << kMaskShift) - 1u;
constexpr int kBlendThreads = 64;     // one wave per 16x16 tile, four pixels per thread (blend)
constexpr int kBlendBatch = 128;      // Gaussians staged in LDS per step (blend)
constexpr int kBlendRun = 128;        // consecutive tiles one XCD takes in a row (blend)
constexpr int kMaxSeg = 16;           // (viewer, eye) images per raster batch
constexpr int kGridBlocks = 2048;     // fixed grid of the grid-stride kernels
constexpr int kScanBlocks = 1024;     // blocks of the device-wide scan
constexpr int kSortBlocks = 1024;     // blocks of each radix pass
constexpr int kF = 32;                // feature length the kernels are built for
constexpr int kH = 32;                // MLP hidden width the kernels are built for
constexpr int kMaxK = 16;             // max neural Gaussians per anchor
constexpr int kPredW = 64;            // reuse predictor width
constexpr int kPredIn = 6;            // reuse predictor features

// Device counters of one view (viewer).  Every frame-dependent size lives
// here so that a frame never waits on the host.
struct Counters {
    int32_t n_visible;
    int32_t n_miss;
    int32_t n_need;      // misses without a line
    int32_t n_free;      // free lines after invalidation
    int32_t n_gauss;
    int32_t n_evict;
    int32_t depth;       // d_t for the next frame to run
    int32_t depth_used;  // d_t applied by the last frame
    int32_t n_cand;      // reuse candidates (predictor inputs)
    int32_t overflow;    // bit1: cache capacity
    int32_t evict_short; // lines still to evict
    int32_t evict_thr;   // last_used threshold of partial eviction bin
    int32_t evict_left;  // evictions taken from the threshold bin
    int32_t pad[3];
};

// Device counters of one raster batch.
struct RasterCounters {
    int32_t n_entries;            // total (segment, Gaussian) entries
    int32_t entry_base[kMaxSeg + 1];  // entry of Gaussian 0 of each segment (total last)
    int32_t entry_stride;             // 2 with paired segments, else 1
    int32_t n_pairs;              // total (super tile, entry) pairs (all segments): the sorted items
    int32_t n_echunks;            // chunks of 256 entries (preprocess tall lists)
    int32_t n_tall_e;             // tall entries found by the preprocess
    int32_t n_srows;              // their super rows (pairs of tile rows), stored
    int32_t overflow;             // bit0: pair capacity, bit1: entries, bit2: tall footprints' super rows
    int32_t n_gpairs;             // entries / 2: the depth sort's length when the eyes share it
};

// One (viewer, eye) image of a raster batch; passed by value in kernel args.
struct Seg {
    const float4* L0;   // mu - anchor (xyz), alpha   [entries of the view's cache]
    const float4* L1;   // cov xx xy xz yy
    const float4* L2;   // cov yz zz, r, g
    const float* L3;    // b
    const int32_t* G;   // render buffer: cache entry per Gaussian (nullptr = identity)
    const int32_t* nG;  // device count of G (nullptr = nG_host)
    int32_t nG_host;
    const float4* anchor_pos;    // anchors (x, y, z, radius); nullptr: L0 holds absolute positions
    const int32_t* line_anchor;  // anchor of each cache line (nullptr: line i belongs to anchor i)
    int32_t k;                   // entries per cache line
    int32_t W, H, ntx, nty;
    int32_t tile_base;  // first global tile id of this image
    int32_t sup_base;   // first global super-tile id of this image (set by raster_batch)
    int32_t nsx, nsy;   // super tiles per row and column
    float R[9];
    double pos[3];      // eye position (FP64: subtracted from FP32 anchor positions)
    float fx, fy, cx, cy, limx, limy, znear;
    float* out_rgb;     // [3,H,W]
    float* out_T;       // [H,W] or nullptr
    int32_t* out_nc;    // [H,W] or nullptr
    // fractional level transition (nullptr level: off): opacities of a
    // level-l anchor's Gaussians scaled by clamp(2 - |x - p_u| / d_l, 0, 1)
    const uint8_t* level;
    float upos[3];      // unified camera centre p_u (as the selection uses it)
    float d_ref;
};

// paired: segments 2p and 2p+1 are the two eyes of one view (the same render
// buffer and cache lines), and their entries interleave, entry = base_p +
// 2 g + eye, so both eyes of a Gaussian are projected by neighbouring lanes
// from one read of its line; otherwise segment q's entries are contiguous.
struct SegTable {
    int32_t n;
    int32_t total_tiles;
    int32_t paired;
    int32_t total_sup;  // super tiles of all images (set by raster_batch)
    Seg s[kMaxSeg];
};

// Unified-camera constants for the derive stage (FP32, computed in FP64).
struct DeriveCam {
    float pos[3];        // p_u
    float planes[5][4];  // inward world planes n.x + w >= -radius keeps
    float d_ref;
    float fx;            // unified focal length (predictor feature)
    int32_t fade;        // fractional level transition: keep level l > 0 while |x - p_u| < 2 d_l
};

// Scene on the device (shared by views).
struct Scene {
    int64_t n = 0;
    int k = 0;
    float d_ref = 0.f;
    float dist_unit = 0.f;      // > 0: the MLPs' distance input is |x - p_u| / dist_unit
    int l_max = 0;
    float4* posr = nullptr;     // x, y, z, radius
    uint8_t* level = nullptr;
    float* feat = nullptr;      // [n, F]
    float* scale = nullptr;     // [n, 6]
    float* offsets = nullptr;   // [n, k, 3]
    // MFMA weight fragments (see gsc_derive_mfma.h)
    float* fr_l1_f32 = nullptr;
    float* fr_l2_f32 = nullptr;
    uint16_t* fr_l1_bf16 = nullptr;
    uint16_t* fr_l2_bf16 = nullptr;
    uint16_t* fr_l1_fp8 = nullptr;
    uint16_t* fr_l2_fp8 = nullptr;
    float* fr_b1 = nullptr;
    float* fr_b2 = nullptr;
    float* fr_s1 = nullptr;
    float* fr_s2 = nullptr;
    int n_at = 0, n_ct = 0, n_vt = 0;
    size_t bytes = 0;
};

// Per-viewer derive state: cache lines and the render buffer.
struct View {
    int64_t C = 0;              // cache lines
    int64_t max_gauss = 0;
    int32_t* slot_of = nullptr; // [n] line of each anchor or -1
    int32_t* line_anchor = nullptr, *line_tau = nullptr, *line_last = nullptr;  // [C]
    float4* L0 = nullptr, *L1 = nullptr, *L2 = nullptr;  // [C*k]
    uint16_t* line_mask = nullptr;  // [C] bit j: entry j of the line has alpha > 0
    float* L3 = nullptr;
    float* pu_hist = nullptr;   // [64][4] unified camera centre per frame (t mod 64)
    int32_t* visible = nullptr; // [n]
    int32_t* vslot = nullptr;   // [n] line per visible position
    uint32_t* tmp_a = nullptr;  // [max(n, C)] scratch
    uint32_t* tmp_b = nullptr;  // [max(n, C)] scratch
    uint32_t* tmp_c = nullptr;  // [max(n, C)] scratch
    uint32_t* tmp_d = nullptr;  // [max(n, C)] scratch
    uint32_t* evict_hist = nullptr;  // [64]
    int32_t* evict_scan_n = nullptr; // [1] count for the eviction scans
    int32_t* misses = nullptr;  // [n] visible positions of misses
    int32_t* free_list = nullptr; // [C]
    int32_t* G = nullptr;       // [max_gauss]
    uint32_t* block_sums = nullptr;  // scan scratch
    float* cand_feat = nullptr; // [n, 6] predictor features
    int32_t* cand_id = nullptr; // [n]
    Counters* cnt = nullptr;
    Counters* cnt_host = nullptr;  // pinned mirror
    int64_t t = 0;
    size_t bytes = 0;
};

// A tall footprint (more than four tile rows) as the span kernel reads it:
// its ellipse (the conic, opacity-aware threshold and the extents the row
// spans start from), entry, tile rows and segment.
struct TallRec {
    float mx, my, ca, cb, cc, tau, det, xmax, ymax, kr, margin, ia, ic;
    uint32_t e, rows, seg;
};
static_assert(sizeof(TallRec) == 64, "tall footprint record: four 16-byte words");

// Raster batch buffers.
struct Raster {
    int64_t max_entries = 0, max_pairs = 0, max_tiles = 0;
    float4* rec = nullptr;      // [4 * entries]: (mean2d, conic a b), (conic c, alpha, r g), (b, rows, seg, count),
                                // spans (tall footprints: first stored span, output offset)
    int32_t* pt_list = nullptr;   // [max_entries] tall entries (entry ids) in their chunk's slots
    uint64_t* pt_pack = nullptr;  // [max_entries / 256 + 1] per chunk of entries: tall ones | their super rows << 32
    uint64_t* pt_off = nullptr;   // [max_entries / 256 + 1] exclusive prefix of pt_pack
    TallRec* trec = nullptr;  // [tall_cap] the tall footprints (ellipse, entry, rows, segment), dense
    uint32_t* pt_sroff = nullptr;  // [tall_cap] first stored super row of each
    int64_t tall_cap = 0;
    uint4* srow = nullptr;        // [srow_cap] super rows of the tall footprints: span of tile row 2 Y,
                                  // of tile row 2 Y + 1 (lo | hi << 16), entry, items of the earlier ones
    int32_t* srow_y = nullptr;    // [srow_cap] Y of each stored super row
    int64_t srow_cap = 0;
    uint32_t* ntiles = nullptr; // tile count per entry
    uint32_t* nsup = nullptr;   // (super tile, entry) pair count per entry
    uint32_t* scnt = nullptr;   // pair count per depth rank
    int32_t* n_sort = nullptr;  // [1] pairs to sort (clamped to capacity)
    uint32_t* dkey[2] = {nullptr, nullptr};  // depth keys (double buffer)
    uint32_t* dval[2] = {nullptr, nullptr};  // entry ids
    uint32_t* offs = nullptr;   // pair offset per depth rank
    int32_t* tile_eval = nullptr;  // [max_tiles][2] blend visits and contributions of each tile
    uint32_t* pkey[2] = {nullptr, nullptr};  // global tile id
    uint32_t* pval[2] = {nullptr, nullptr};  // entry id
    uint64_t* pkey64[2] = {nullptr, nullptr};// full-key mode
    int32_t* ranges = nullptr;  // [max_tiles][2]
    uint32_t* hist = nullptr;   // [256 * kSortBlocks] radix digit counts per block
    uint32_t* block_sums = nullptr;
    uint64_t* block_sums64 = nullptr;  // [kScanBlocks] scan scratch of the tall path's 64-bit scan
    RasterCounters* cnt = nullptr;
    RasterCounters* cnt_host = nullptr;
    int sorted_buf = 0;         // which pkey/pval buffer holds the sorted pairs
    bool key16 = false;         // the last batch's tile keys were 16-bit (pkey read as uint16_t)
    bool shared_depth = false;  // this batch's eyes of a view share one depth sort
    const uint32_t* order = nullptr;  // depth rank -> entry (null: pair values are entries)
    size_t bytes = 0;
};

// ----------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns hipSuccess or the launch error.

// Device-wide exclusive scan of n uint32 values (n from *n_dev if non-null),
// writing exclusive prefixes to out and the total to *total (device).
hipError_t scan_u32(const uint32_t* in, uint32_t* out, const int32_t* n_dev, int64_t n_host, int32_t* total,
                    uint32_t* block_sums, hipStream_t st);
// Exclusive scan of n (from *n_dev) uint64 values, each two 32-bit counts
// (low, high) that scan independently; the totals of the two go to
// *total_lo and *total_hi (device).  block_sums: kScanBlocks values.
hipError_t scan_u64(const uint64_t* in, uint64_t* out, const int32_t* n_dev, int32_t* total_lo, int32_t* total_hi,
                    uint64_t* block_sums, hipStream_t st);
// Stream compaction: ids[k] = the k-th i with flags[i] != 0 (flags 0 or 1,
// n from *n_dev if non-null), the count to *total (device).
hipError_t compact_u32(const uint32_t* flags, const int32_t* n_dev, int64_t n_host, int32_t* total, int32_t* ids,
                       uint32_t* block_sums, hipStream_t st);

// Stable LSD radix sort of (key, value) pairs over bits [bit0, bit1),
// 8-bit digits, reduce-then-scan per pass (digit counts per block, a scan of
// the counts in digit-major order, a scatter through LDS).  Count from
// *n_dev (device) or n_host.  Returns in *which the buffer index (0/1)
// holding the result.  hist: [256 * kSortBlocks], block_sums: scan scratch.
// With gout, the last pass writes gout[i] = gsrc[sorted value i] in place of
// the sorted keys (which are then not produced).  With gout and pairs, each
// value v stands for the two elements 2v, 2v+1: the last pass writes, for
// sorted position i, vals[2i + h] = 2v + h and gout[2i + h] = gsrc[2v + h]
// (h = 0, 1), so the result holds 2n values (the value buffers must hold
// them).
hipError_t radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], const int32_t* n_dev, int64_t n_host, int bit0,
                          int bit1, uint32_t* hist, uint32_t* block_sums, int* which, hipStream_t st,
                          const uint32_t* gsrc = nullptr, uint32_t* gout = nullptr, bool pairs = false);
hipError_t radix_sort_u64(uint64_t* keys[2], uint32_t* vals[2], const int32_t* n_dev, int64_t n_host, int bit0,
                          int bit1, uint32_t* hist, uint32_t* block_sums, int* which, hipStream_t st);
// 16-bit keys (tile ids of batches with at most 65,536 tiles).
hipError_t radix_sort_u16(uint16_t* keys[2], uint32_t* vals[2], const int32_t* n_dev, int64_t n_host, int bit0,
                          int bit1, uint32_t* hist, uint32_t* block_sums, int* which, hipStream_t st);




// Derive stage of one view.
struct DeriveArgs {
    const Scene* sc;
    View* v;
    DeriveCam cam;
    int precision;
    uint32_t flags;
    int d_max;
    int guide;
    float pred_thr;
    const float* pred_w;      // predictor params (device fp32)
    const uint16_t* pred_wbf; // bf16 copy for inference
    int collect;              // store reuse-candidate features for label collection
};
// Optional stage timing: HIP events recorded on the stream at the stage
// boundaries of one frame (GSC_STAGE_* order of the public header).
constexpr int kNumStages = 13;
struct Marks {
    hipEvent_t ev[kNumStages + 1];
    uint32_t recorded;  // bit i: ev[i] recorded this frame
    uint32_t want;      // bit i: record ev[i]
};
inline void mark(Marks* m, int i, hipStream_t st) {
    if (m && (m->want >> i & 1u) && hipEventRecord(m->ev[i], st) == hipSuccess) m->recorded |= 1u << i;
}

hipError_t derive_frame(const DeriveArgs& a, hipStream_t st, Marks* mk = nullptr);

// Mean SSIM (gsc_metrics.hip): the normalised 11-tap Gaussian window, the
// number of per-block partial sums for C channels of H x W (H, W >= 11),
// and the launch writing the partials and their total (the sum of the map
// over every window position and channel) on the device.
struct SsimWindow {
    double w[11];
};
SsimWindow ssim_window();
int64_t ssim_blocks(int C, int H, int W);
hipError_t ssim_launch(const float* a, const float* b, int C, int H, int W, const SsimWindow& win, double* partial,
                       double* total, hipStream_t st);

// Raster stage of a batch of segments.
// count_work: the blend also counts its (pixel, Gaussian) visits and
// contributions per tile (and writes per-pixel contributor counts when a
// segment asks for them); without it those counters are not kept.
// blend_st (optional): the stream the blend runs on, after front_done is
// recorded on st once the tile ranges are written (the stage marks of the
// blend go to blend_st as well).
hipError_t raster_batch(const SegTable& tab, Raster& r, bool full_key_sort, bool count_work, hipStream_t st,
                        Marks* mk = nullptr, hipStream_t blend_st = nullptr, hipEvent_t front_done = nullptr);

// Blocks of `threads` threads of `kernel` the whole device holds at once
// (occupancy x compute units; cached per kernel and device).  Grid-stride
// kernels launch at most this many, so that no block waits for a second
// round while the rest of the chip idles.
int resident_blocks(const void* kernel, int threads);

// Grid of a grid-stride kernel over n items, one item per thread per step.
template <typename K>
inline dim3 grid_fit(K* kernel, int64_t n, int threads = 256) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    const int64_t cap = resident_blocks((const void*)kernel, threads);
    return dim3((unsigned)(b < cap ? b : cap));
}

// Fill a segment's camera fields from a public camera.
void seg_camera(Seg& s, const gsc_camera& c);
// Super-tile geometry of every segment (sup_base, nsx, nsy) and the total,
// from the segments' tile grids, in segment order.
void seg_supers(SegTable& tab);

// Predictor kernels.
hipError_t pred_forward_bwd(const float* w, const float* X, const float* y, int n, float pos_weight, float* grads,
                            float* loss, hipStream_t st);
hipError_t pred_adam(float* w, const float* grads, float* m, float* v, int nparams, int step, float lr,
                     hipStream_t st);
hipError_t pred_infer(const uint16_t* wbf, const float* w32, const float* X, int n, float* p, hipStream_t st);
hipError_t pred_to_bf16(const float* w, uint16_t* wbf, int n, hipStream_t st);

}  // namespace gsc
