// Raster stage (Section 3.1 splatting + Section 6 RasterizeGaussians) for a
// batch of images ("segments": one per (viewer, eye)), all in one set of
// launches:
//   k_preprocess       EWA projection, conic, opacity-aware extent, depth
//                      key, exact tile spans of footprints up to 4 tile
//                      rows (per entry); segment bases; clears the ranges
//   tall spans         the taller footprints' super rows (pairs of tile rows),
//                      a group of lanes per footprint, one tile row per lane
//   depth radix pass   stable sort of entries by float32 depth (the low 32
//                      bits of the (tile | depth) key, applied per Gaussian
//                      before duplication); the last pass also lays the tile
//                      counts out in depth order.  When a view's two eyes
//                      share its rotation, one key per Gaussian orders both
//                      eyes' entries (half the keys)
//   scan + k_dup_rows / k_dup_big
//                      one (global super-tile id, entry | tile mask) item per
//                      covered super tile (2x2 tiles), emitted in depth order
//   super-tile radix pass
//                      stable sort of the items by global super-tile id
//   k_ranges           [start, end) of every super tile's run
//   k_blend            front-to-back compositing, one launch over every
//                      (segment, tile) of the batch, one block per 16x16
//                      tile (interleaved tile runs per XCD); a tile stages the
//                      entries of its super tile's list that carry its mask
//                      bit, LDS batches, block-wide early exit
// With full_key_sort the items carry the whole 64-bit (super tile << 32 |
// depth) key and are sorted after duplication instead; the order is the same.
#include <cmath>
#include <cstring>

#include "gsc_blockscan.h"
#include "gsc_common.h"

namespace gsc {

namespace {

constexpr int NT = 256;
constexpr float kMinAlpha = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;

__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }


// Segment -> entry of its Gaussian 0, from the segments' device counts
// (every block of k_preprocess computes it; block 0 publishes it for the
// later kernels); base[n] is the total.  Paired segments interleave: the
// pair's base, +1 for the second eye, stride 2.
__device__ __forceinline__ int32_t seg_count(const Seg& s) { return s.nG ? *s.nG : s.nG_host; }

__device__ __forceinline__ int32_t entry_bases(const SegTable& tab, int64_t max_entries, int32_t* base,
                                               bool& over) {
    int32_t acc = 0;
    if (tab.paired) {
        for (int q = 0; q + 1 < tab.n; q += 2) {
            base[q] = acc;
            base[q + 1] = acc + 1;
            acc += 2 * seg_count(tab.s[q]);
        }
    } else {
        for (int q = 0; q < tab.n; ++q) {
            base[q] = acc;
            acc += seg_count(tab.s[q]);
        }
    }
    base[tab.n] = acc;
    over = acc > max_entries;
    // (paired: whole pairs only, so both eyes' entries of a Gaussian stay together)
    return over ? (int32_t)(tab.paired ? (max_entries & ~(int64_t)1) : max_entries) : acc;
}

// Entry e -> (segment si, Gaussian g of that segment).
__device__ __forceinline__ void locate_entry(const SegTable& tab, const int32_t* base, int64_t e, int& si,
                                             int64_t& g) {
    si = 0;
    if (tab.paired) {
        while (si + 2 < tab.n && e >= base[si + 2]) si += 2;
        const int64_t off = e - base[si];
        si += (int)(off & 1);
        g = off >> 1;
    } else {
        while (si + 1 < tab.n && e >= base[si + 1]) ++si;
        g = e - base[si];
    }
}

// Minimum of q(d) = a dx^2 + 2 b dx dy + c dy^2 over the closed rectangle
// [x0,x1] x [y0,y1] of offsets d (q convex: 0 inside, else on an edge; the
// edge minimiser of a 1-D quadratic, clamped).  ia = 1/a, ic = 1/c.
// Every footprint's tile spans are computed once (here or in k_tall_spans)
// and stored, so counting and emission read the same decisions.
// Minimum over the vertical edge x = dx and the horizontal edge y = ey.
__device__ __forceinline__ float edge_min_q(float a, float b, float c, float ia, float ic, float x0, float x1,
                                            float y0, float y1, float dx, float ey) {
    float dy = fminf(fmaxf(-b * dx * ic, y0), y1);
    float ex = fminf(fmaxf(-b * ey * ia, x0), x1);
    return fminf(a * dx * dx + 2.f * b * dx * dy + c * dy * dy, a * ex * ex + 2.f * b * ex * ey + c * ey * ey);
}

// kRolled keeps the two edge pairs in a loop: unrolled, the compiler keeps
// both pairs' terms of every inlined call live at once, which costs
// k_preprocess (one footprint per lane, many rows) about 60 VGPRs; the tall
// kernel (one row per lane, a serial tile scan) runs faster unrolled.
template <bool kRolled>
__device__ __forceinline__ float rect_min_q(float a, float b, float c, float ia, float ic, float x0, float x1,
                                            float y0, float y1) {
    if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return 0.f;
    float best = INFINITY;
    float fx[2] = {x0, x1}, fy[2] = {y0, y1};
    if constexpr (kRolled) {
#pragma unroll 1
        for (int i = 0; i < 2; ++i) best = fminf(best, edge_min_q(a, b, c, ia, ic, x0, x1, y0, y1, fx[i], fy[i]));
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) best = fminf(best, edge_min_q(a, b, c, ia, ic, x0, x1, y0, y1, fx[i], fy[i]));
    }
    return best;
}

// Exact tile span of one tile row.  The footprint E = {q <= tau} meets the
// pixel-centre rectangle of a tile iff the x-extent of E inside the row's
// pixel-centre band overlaps the tile's x-span; the tiles hit in a row are
// therefore contiguous.  The extent is computed analytically; tiles clearly
// inside it (by a margin far above FP32 error) are hit, tiles near its ends
// get the exact rectangle test.
struct Ellipse {
    float mx, my, ca, cb, cc, tau;
    float det, xmax, ymax, kr;  // kr: dy of the rightmost point is -cb * kr
    float margin;
    float ia, ic;               // 1/ca, 1/cc
};

// The extents (xmax, ymax, kr, and the row extents below) only place the
// candidate range and the certain interior, each widened by the margin, which
// is far above the 1-ulp error of the hardware square root and reciprocal;
// ia and ic enter the exact test and stay correctly rounded.
__device__ __forceinline__ Ellipse make_ellipse(float mx, float my, float ca, float cb, float cc, float tau) {
    Ellipse e;
    e.mx = mx; e.my = my; e.ca = ca; e.cb = cb; e.cc = cc; e.tau = tau;
    e.det = ca * cc - cb * cb;
    e.ia = 1.0f / ca;
    e.ic = 1.0f / cc;
    const float id = e.det > 0.f ? __builtin_amdgcn_rcpf(e.det) : 0.f;
    e.xmax = __builtin_amdgcn_sqrtf(tau * cc * id);
    e.ymax = __builtin_amdgcn_sqrtf(tau * ca * id);
    e.kr = __builtin_amdgcn_sqrtf(tau * id * e.ic);
    e.margin = 2e-3f * (e.xmax + e.ymax) + 0.05f;
    return e;
}

// Does the footprint reach the pixel-centre rectangle of tile (tx, ty)?
template <bool kRolled>
__device__ __forceinline__ bool tile_hit(const Ellipse& e, int tx, int ty, int W, int H) {
    float x0 = (float)(kTile * tx) + 0.5f, y0 = (float)(kTile * ty) + 0.5f;
    float x1 = (float)min(kTile * tx + kTile - 1, W - 1) + 0.5f;
    float y1 = (float)min(kTile * ty + kTile - 1, H - 1) + 0.5f;
    return rect_min_q<kRolled>(e.ca, e.cb, e.cc, e.ia, e.ic, x0 - e.mx, x1 - e.mx, y0 - e.my, y1 - e.my) <= e.tau;
}

template <bool kRolled>
__device__ __forceinline__ void row_span(const Ellipse& e, int ty, int ntx, int W, int H, int& lo, int& hi) {
    lo = 0;
    hi = -1;
    const float y0 = (float)(kTile * ty) + 0.5f - e.my;
    const float y1 = (float)min(kTile * ty + kTile - 1, H - 1) + 0.5f - e.my;
    if (y0 > e.ymax + e.margin || y1 < -e.ymax - e.margin) return;  // band clear of E
    float L, R;       // x-extent of E inside the band (offsets from mx)
    bool certain;     // extent reliable enough to classify interior tiles
    const float b0 = fmaxf(y0, -e.ymax), b1 = fminf(y1, e.ymax);
    if (b0 > b1) {
        // The band lies beyond a tip of E, within the margin: E can reach it
        // only near that tip, so the exact test decides over a short range.
        // The chords of E at |dy| >= d1 lie inside the chord at d1 (they
        // shrink towards the tip) shifted by at most |cb| / ca per unit of
        // dy (their centres move along dx = -cb dy / ca) over the rest of
        // the way to the tip, which is less than ymax - d1 + margin.
        const float d1 = fmaxf(e.ymax - e.margin, 0.f);
        const float dy1 = y0 > 0.f ? d1 : -d1;
        const float s1 = __builtin_amdgcn_sqrtf(fmaxf(e.ca * e.tau - e.det * dy1 * dy1, 0.f));
        const float cen = -e.cb * dy1 * e.ia;
        const float wid = s1 * e.ia + fabsf(e.cb) * e.ia * (e.ymax - d1 + e.margin);
        L = cen - wid;
        R = cen + wid;
        certain = false;
    } else {
        float dyr = fminf(fmaxf(-e.cb * e.kr, b0), b1);
        float dyl = fminf(fmaxf(e.cb * e.kr, b0), b1);
        float sr = __builtin_amdgcn_sqrtf(fmaxf(e.ca * e.tau - e.det * dyr * dyr, 0.f));
        float sl = __builtin_amdgcn_sqrtf(fmaxf(e.ca * e.tau - e.det * dyl * dyl, 0.f));
        R = (-e.cb * dyr + sr) * e.ia;
        L = (-e.cb * dyl - sl) * e.ia;
        certain = true;
    }
    const float m = e.margin;
    // tile tx spans x in [16 tx + 0.5, 16 tx + 15.5] (clipped at the image edge)
    float ca_lo = ceilf((e.mx + L - m - 15.5f) * (1.0f / kTile));
    float ca_hi = floorf((e.mx + R + m - 0.5f) * (1.0f / kTile));
    int c_lo = (int)fminf(fmaxf(ca_lo, 0.f), (float)ntx);
    int c_hi = (int)fminf(fmaxf(ca_hi, -1.f), (float)(ntx - 1));
    if (c_lo > c_hi) return;
    int s_lo = c_hi + 1, s_hi = c_hi;  // certain interior [s_lo, s_hi]
    if (certain && R - L > 2.f * m) {
        float sa = ceilf((e.mx + L + m - 15.5f) * (1.0f / kTile));
        float sb = floorf((e.mx + R - m - 0.5f) * (1.0f / kTile));
        int last_full = (W % kTile) ? ntx - 2 : ntx - 1;  // a clipped last tile is always tested
        s_lo = (int)fminf(fmaxf(sa, (float)c_lo), (float)(c_hi + 1));
        s_hi = (int)fminf(fmaxf(sb, (float)(s_lo - 1)), (float)min(c_hi, last_full));
    }
    const bool has_s = s_lo <= s_hi;
    // Exact tests: from the left over [c_lo, lim] up to the first hit l
    // (none: the interior's first tile, or no tile at all without an
    // interior), then from the right over [stop, c_hi] down to the first hit
    // (none: the interior's last tile, or l, which is hit).  One loop runs
    // both scans, one test a trip, so a wave pays for the most tests any of
    // its lanes needs rather than for its longest left scan plus its longest
    // right scan.
    const int lim = has_s ? s_lo - 1 : c_hi;
    int l = s_lo, h = s_hi, stop = s_hi + 1;
    int tx = c_lo;
    bool left = true, done = false;
    if (lim < c_lo) {  // nothing to test on the left (then there is an interior)
        left = false;
        tx = c_hi;
        done = tx < stop;
    }
    while (!done) {
        const bool hit = tile_hit<kRolled>(e, tx, ty, W, H);
        if (left) {
            if (hit || tx == lim) {
                if (!hit && !has_s) return;  // no tile of the row is hit
                if (hit) l = tx;
                left = false;
                if (!has_s) {
                    stop = l + 1;
                    h = l;
                }
                tx = c_hi;
                done = tx < stop;
            } else {
                ++tx;
            }
        } else {
            if (hit) {
                h = tx;
                done = true;
            } else {
                --tx;
                done = tx < stop;
            }
        }
    }
    lo = l;
    hi = h;
}

// Exclusive scan over one wave64 (total in `total`).
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
    const int lane = threadIdx.x & 63;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

__device__ __forceinline__ Ellipse shfl_ellipse(const Ellipse& el, int src) {
    Ellipse eb;
    eb.mx = __shfl(el.mx, src, 64); eb.my = __shfl(el.my, src, 64);
    eb.ca = __shfl(el.ca, src, 64); eb.cb = __shfl(el.cb, src, 64); eb.cc = __shfl(el.cc, src, 64);
    eb.tau = __shfl(el.tau, src, 64); eb.det = __shfl(el.det, src, 64);
    eb.xmax = __shfl(el.xmax, src, 64); eb.ymax = __shfl(el.ymax, src, 64);
    eb.kr = __shfl(el.kr, src, 64); eb.margin = __shfl(el.margin, src, 64);
    eb.ia = __shfl(el.ia, src, 64); eb.ic = __shfl(el.ic, src, 64);
    return eb;
}

// Footprints taller than this many tile rows get one thread per row for
// their spans (k_tall_spans) and are emitted by super rows (k_dup_big); shorter
// ones keep their row spans in the record and are emitted from them.
constexpr int kSmallRows = 4;

// Fractional level transition: weight clamp(2 - |x - p_u| / d_l, 0, 1) of a
// level-l anchor's opacities (1 at level 0), the distance taken in FP32 as
// the selection takes it.
__device__ __forceinline__ float lod_fade_weight(float4 ap, int l, const Seg& s) {
    if (l == 0) return 1.f;
    const float vx = ap.x - s.upos[0], vy = ap.y - s.upos[1], vz = ap.z - s.upos[2];
    const float d = sqrtf(vx * vx + vy * vy + vz * vz);
    return fminf(fmaxf(2.f - d / ldexpf(s.d_ref, -l), 0.f), 1.f);
}

// Span word of a tile row: lo | hi << 16, hi < lo (0xffff, 0) when empty.
__device__ __forceinline__ int span_lo(uint32_t sp) { return (int)(sp & 0xffffu); }
__device__ __forceinline__ int span_hi(uint32_t sp) { return (int)(sp >> 16); }

// Super-tile columns [x0, x1] of a super row from the spans of its two tile
// rows a (even) and b (odd), either possibly empty: the hull of the rows'
// super columns (a convex footprint's rows give adjacent or overlapping
// ranges; a column of the hull whose mask is empty is emitted with mask 0,
// which no tile reads).  Returns the column count (0: both rows empty).
__device__ __forceinline__ uint32_t sup_cols(uint32_t sa, uint32_t sb, int& x0) {
    int lo = 0x7fffffff, hi = -1;
    if (span_hi(sa) >= span_lo(sa)) { lo = span_lo(sa) >> kSupShift; hi = span_hi(sa) >> kSupShift; }
    if (span_hi(sb) >= span_lo(sb)) {
        lo = min(lo, span_lo(sb) >> kSupShift);
        hi = max(hi, span_hi(sb) >> kSupShift);
    }
    x0 = lo;
    return hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
}

// Mask of the tiles of super column x covered by tile rows a and b: bit
// 2 (ty & 1) + (tx & 1).
__device__ __forceinline__ uint32_t sup_mask(uint32_t sa, uint32_t sb, int x) {
    const int t0 = x << kSupShift, t1 = t0 + 1;
    const int la = span_lo(sa), ha = span_hi(sa), lb = span_lo(sb), hb = span_hi(sb);
    return (uint32_t)(la <= t0 && t0 <= ha) | ((uint32_t)(la <= t1 && t1 <= ha) << 1) |
           ((uint32_t)(lb <= t0 && t0 <= hb) << 2) | ((uint32_t)(lb <= t1 && t1 <= hb) << 3);
}

constexpr uint32_t kEmptySpan = 0x0000ffffu;

// Super pairs of a footprint of at most kSmallRows tile rows from y0 (row i
// at y0 + i, empty rows past the footprint): its super rows are the pairs
// (2 Y, 2 Y + 1) of tile rows.
__device__ __forceinline__ uint32_t small_sup_count(const uint32_t (&sp)[4], int y0) {
    uint32_t n = 0;
    // super row of row 0 holds rows 0 and 1 when y0 is even, row 0 alone (as
    // its row b) when y0 is odd; then rows (1, 2) or (2, 3), and so on
    const int odd = y0 & 1;
    int x0;
    n += sup_cols(odd ? kEmptySpan : sp[0], odd ? sp[0] : sp[1], x0);
    n += sup_cols(odd ? sp[1] : sp[2], odd ? sp[2] : sp[3], x0);
    if (odd) n += sup_cols(sp[3], kEmptySpan, x0);
    return n;
}

// Per-entry record, 4 x float4 (64 B, one cache line):
//   A = (mean2d.x, mean2d.y, conic a, conic b)
//   B = (conic c, alpha, r, g)
//   C = (b, bits: tile rows y0 | y1 << 16, bits: segment, bits: (super tile, entry) pair count)
//   D = bits: exact tile span lo | hi << 16 of each of up to kSmallRows rows
//       (footprints of at most kSmallRows tile rows; hi < lo: empty row)
constexpr int kRec = 4;
struct PreArgs {
    SegTable tab;
    RasterCounters* rc;
    float4* rec;
    uint32_t* ntiles;
    uint32_t* nsup;
    uint32_t* dkey;
    uint32_t* dval;
    int32_t* tall_list;   // tall entries of each chunk of 256 entries, in the chunk's slots
    uint64_t* tall_pack;  // per chunk: its tall entries | their super rows << 32
    int32_t* ranges;     // [2 * tiles] cleared here for this batch's ranges
    int64_t n_ranges;
    int64_t max_entries;
    int32_t shared_depth;  // paired eyes of one rotation: one depth key per Gaussian
};

// (at most 72 VGPRs, no spill: seven waves per SIMD to cover the chain of
// dependent loads of an entry)
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(7))) void k_preprocess(PreArgs p) {
    __shared__ uint32_t s_wtall[NT / 64];
    __shared__ uint32_t s_srows;  // super rows of the step's tall footprints
    // the block's records, copied out together once complete (whole lines,
    // coalesced: a record written in two halves far apart in time would
    // leave half-written lines for the L2 to evict)
    __shared__ float4 s_rec[NT * kRec];
    __shared__ int32_t s_base[kMaxSeg + 1];
    __shared__ int32_t s_ne;
    if (threadIdx.x == 0) {
        bool over;
        s_ne = entry_bases(p.tab, p.max_entries, s_base, over);
        if (blockIdx.x == 0) {  // this batch's counters, for the later kernels
            for (int q = 0; q <= p.tab.n; ++q) p.rc->entry_base[q] = s_base[q];
            p.rc->entry_stride = p.tab.paired ? 2 : 1;
            p.rc->overflow = over ? 2 : 0;
            p.rc->n_entries = s_ne;
            p.rc->n_gpairs = s_ne >> 1;
            p.rc->n_echunks = (s_ne + NT - 1) / NT;
        }
    }
    if (threadIdx.x == 0) s_srows = 0u;
    for (int64_t i = gtid(); i < p.n_ranges; i += gstride()) p.ranges[i] = 0;
    __syncthreads();
    const int64_t ne = s_ne;
    const int lane = threadIdx.x & 63;
    // block-uniform loop: each step covers one chunk of 256 entries, whose
    // tall footprints the block lists together
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < ne; base += gstride()) {
        const int64_t e = base + threadIdx.x;
        const bool valid = e < ne;
        int si = 0;
        uint32_t count = 0, scount = 0, rows = 0;
        float depth = 0.f;
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = make_float4(0.f, 0.f, 0.f, 0.f);
        float lb = 0.f;
        Ellipse el{};
        int y0 = 0, y1 = -1;
        uint32_t spans[kSmallRows] = {0xffffu, 0xffffu, 0xffffu, 0xffffu};
        if (valid) {
            int64_t g;
            locate_entry(p.tab, s_base, e, si, g);
            const Seg& s = p.tab.s[si];
            int64_t src = s.G ? (int64_t)s.G[g] : g;
            float4 l0 = s.L0[src], l1 = s.L1[src], l2 = s.L2[src];
            lb = s.L3[src];
            // mu - eye = (anchor - eye) + (mu - anchor): the first term in FP64
            // from the exact FP32 anchor, the second as stored
            double ax = 0.0, ay = 0.0, az = 0.0;
            float lod_w = 1.f;
            if (s.anchor_pos) {
                const int32_t an = s.line_anchor ? s.line_anchor[src / s.k] : (int32_t)(src / s.k);  // valid for every line in the buffer
                const int32_t ai = an >= 0 ? an : 0;
                const float4 ap = s.anchor_pos[ai];
                ax = ap.x; ay = ap.y; az = ap.z;
                if (s.level) lod_w = lod_fade_weight(ap, s.level[ai], s);
            }
            float vx = (float)((ax - s.pos[0]) + (double)l0.x);
            float vy = (float)((ay - s.pos[1]) + (double)l0.y);
            float vz = (float)((az - s.pos[2]) + (double)l0.z);
            float tx = s.R[0] * vx + s.R[1] * vy + s.R[2] * vz;
            float ty = s.R[3] * vx + s.R[4] * vy + s.R[5] * vz;
            float tz = s.R[6] * vx + s.R[7] * vy + s.R[8] * vz;
            float alpha = l0.w * lod_w;
            if (tz > s.znear && alpha >= kMinAlpha) {
                // EWA: Jacobian of the perspective map (off-axis slope clamped)
                float iz = 1.0f / tz;
                float rx = fminf(fmaxf(tx * iz, -s.limx), s.limx);
                float ry = fminf(fmaxf(ty * iz, -s.limy), s.limy);
                float j00 = s.fx * iz, j02 = -s.fx * rx * iz, j11 = s.fy * iz, j12 = -s.fy * ry * iz;
                float T0[3], T1[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T0[k] = j00 * s.R[k] + j02 * s.R[6 + k];
                    T1[k] = j11 * s.R[3 + k] + j12 * s.R[6 + k];
                }
                float S[3][3] = {{l1.x, l1.y, l1.z}, {l1.y, l1.w, l2.x}, {l1.z, l2.x, l2.y}};
                float u0[3], u1[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    u0[r] = S[r][0] * T0[0] + S[r][1] * T0[1] + S[r][2] * T0[2];
                    u1[r] = S[r][0] * T1[0] + S[r][1] * T1[1] + S[r][2] * T1[2];
                }
                float a = T0[0] * u0[0] + T0[1] * u0[1] + T0[2] * u0[2] + 0.3f;
                float b = T0[0] * u1[0] + T0[1] * u1[1] + T0[2] * u1[2];
                float c = T1[0] * u1[0] + T1[1] * u1[1] + T1[2] * u1[2] + 0.3f;
                float det = a * c - b * b;
                if (det > 0.f) {
                    float id = 1.0f / det;
                    float ca = c * id, cb = -b * id, cc = a * id;
                    float mx = s.fx * tx * iz + s.cx, my = s.fy * ty * iz + s.cy;
                    A = make_float4(mx, my, ca, cb);
                    B = make_float4(cc, alpha, l2.z, l2.w);
                    depth = tz;
                    // opacity-aware extent: alpha exp(-q/2) >= 1/255  <=>  q <= 2 ln(255 alpha)
                    float tau = fmaxf(2.0f * logf(255.0f * alpha), 0.f);
                    el = make_ellipse(mx, my, ca, cb, cc, tau);
                    float fy0 = floorf((my - el.ymax - el.margin - 0.5f) * (1.0f / kTile));
                    float fy1 = floorf((my + el.ymax + el.margin - 0.5f) * (1.0f / kTile));
                    y0 = (int)fminf(fmaxf(fy0, 0.f), (float)s.nty);
                    y1 = (int)fminf(fmaxf(fy1, -1.f), (float)(s.nty - 1));
                }
            }
            // the projected record now: its registers are free for the row spans
            s_rec[kRec * threadIdx.x] = A;
            s_rec[kRec * threadIdx.x + 1] = B;
            if (y1 - y0 + 1 <= kSmallRows) {
#pragma unroll
                for (int i = 0; i < kSmallRows; ++i) {
                    int lo = 0xffff, hi = 0;
                    if (y0 + i <= y1) row_span<true>(el, y0 + i, s.ntx, s.W, s.H, lo, hi);
                    if (hi >= lo) count += (uint32_t)(hi - lo + 1);
                    else lo = 0xffff, hi = 0;
                    spans[i] = (uint32_t)lo | ((uint32_t)hi << 16);
                }
                scount = small_sup_count(spans, y0);
            }
        }
        // tall footprints (more than kSmallRows tile rows) are counted later,
        // one thread per row (k_tall_spans); list them in this chunk's slots
        const bool tall = valid && y1 - y0 + 1 > kSmallRows;
        if (valid) {
            rows = y0 <= y1 ? ((uint32_t)y0 | ((uint32_t)y1 << 16)) : 0u;
            s_rec[kRec * threadIdx.x + 2] = make_float4(lb, __uint_as_float(rows), __uint_as_float((uint32_t)si),
                                                        __uint_as_float(scount));
            s_rec[kRec * threadIdx.x + 3] = make_float4(__uint_as_float(spans[0]), __uint_as_float(spans[1]),
                                                        __uint_as_float(spans[2]), __uint_as_float(spans[3]));
            p.ntiles[e] = count;
            p.nsup[e] = scount;
            if (!p.shared_depth) {
                p.dkey[e] = (count || tall) ? __float_as_uint(depth) : 0u;  // tall: settled by k_tall_spans
                p.dval[e] = (uint32_t)e;
            }
        }
        const uint64_t m = __ballot(tall);
        if (lane == 0) s_wtall[threadIdx.x >> 6] = (uint32_t)__popcll(m);
        if (tall) atomicAdd(&s_srows, (uint32_t)((y1 >> kSupShift) - (y0 >> kSupShift) + 1));
        __syncthreads();
        const int64_t chunk = base / NT;
        if (tall) {
            uint32_t at = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            for (int q = 0; q < (int)(threadIdx.x >> 6); ++q) at += s_wtall[q];
            p.tall_list[chunk * NT + at] = (int32_t)e;
        }
        if (threadIdx.x == 0) {
            uint32_t n = 0;
            for (int q = 0; q < NT / 64; ++q) n += s_wtall[q];
            p.tall_pack[chunk] = (uint64_t)n | ((uint64_t)s_srows << 32);
            s_srows = 0u;  // (read above; the next step's adds come after the barrier below)
        }
        {
            const int nv = (int)(ne - base < NT ? ne - base : NT);
            float4* dst = p.rec + kRec * base;
            for (int i = threadIdx.x; i < kRec * nv; i += NT) dst[i] = s_rec[i];
        }
        __syncthreads();  // s_wtall and s_rec are rewritten by the next step
        if (p.shared_depth) {
            // The eyes' entries 2j, 2j+1 sit in neighbouring lanes.  With one
            // rotation for both eyes their view depths differ by a constant,
            // so one key orders both: the left eye's depth when that eye
            // draws the Gaussian, else the right eye's.
            const bool draws = valid && (count || tall);
            const uint32_t mine = draws ? __float_as_uint(depth) : 0u;
            const uint32_t other = (uint32_t)__shfl_xor((int)mine, 1);
            const int odraws = __shfl_xor((int)draws, 1);
            if (valid && !(e & 1)) {
                p.dkey[e >> 1] = draws ? mine : (odraws ? other : 0u);
                p.dval[e >> 1] = (uint32_t)(e >> 1);
            }
        }
    }
}

// Super-tile grid of one segment, as the pair emission needs it.
struct SupGeo {
    int32_t base;  // first global super-tile id
    int32_t nsx;   // super tiles per row
};

struct DupArgs {
    SupGeo sg[kMaxSeg];
    RasterCounters* rc;
    const uint32_t* order;   // depth rank -> entry (depth-presorted mode)
    const uint32_t* offs;    // pair offset per rank (per entry in full-key mode)
    const uint32_t* items;   // item count per rank, the scan's input (an entry without items is skipped unread)
    float4* rec;             // (k_dup_rows stores a tall entry's output offset in D.y)
    const uint32_t* dkey;    // depth key per entry (full-key mode)
    uint32_t* key32;         // global super-tile id (depth-presorted mode, more than 65,536 super tiles)
    uint16_t* key16;         // global super-tile id (depth-presorted mode, at most 65,536 super tiles)
    uint64_t* key64;         // (global super tile << 32 | depth bits) (full-key mode)
    uint32_t* val;           // entry id | tile mask << kMaskShift
    int64_t max_pairs;
    int32_t* n_sort;         // pairs to sort (set by k_dup_rows)
    const uint4* srow;       // super rows of the tall footprints (see k_tall_spans)
    const int32_t* srow_y;   // their super-row index in the image
    int64_t srow_cap;
};

// Kernel arguments (the segment table travels by value) stay within the
// 4 KiB a launch carries.
static_assert(sizeof(PreArgs) <= 4096 && sizeof(DupArgs) + 2 * sizeof(void*) <= 4096,
              "raster kernel arguments exceed 4 KiB");

// Pair emission.  Every entry owns the output range [offs[r], offs[r] +
// count) (ranks in depth order; entry order with full keys), so entries can
// be emitted in any order:
//   k_dup_rows   entries of at most kSmallRows tile rows: the row spans the
//                preprocess stored give each pair's tile; a wave writes its 64
//                entries' pairs together, lane j taking pairs j, j + 64, ...
//                of their concatenation (consecutive lanes, consecutive
//                slots), so the stores coalesce; for a taller entry it
//                stores the output offset in the record instead;
//   k_dup_big    the taller entries' stored rows, 64 to a wave, whatever
//                entries they belong to (below).
template <bool kFull>
__device__ __forceinline__ void put_pair(const DupArgs& d, int64_t q, uint32_t t, uint32_t e, uint64_t low) {
    if (q >= d.max_pairs) return;
    if (kFull) d.key64[q] = ((uint64_t)t << 32) | low;
    else if (d.key16) d.key16[q] = (uint16_t)t;
    else d.key32[q] = t;
    d.val[q] = e;
}

// Pairs to sort (clamped to the capacity; overflow flagged); run by one
// thread of k_dup_rows.
__device__ __forceinline__ void pairs_clamp(RasterCounters* rc, int32_t* n_sort, int64_t max_pairs) {
    int32_t n = rc->n_pairs;
    if ((int64_t)n > max_pairs) {
        rc->overflow |= 1;
        n = (int32_t)max_pairs;
    }
    *n_sort = n;
}

template <bool kFull>
__global__ __launch_bounds__(NT) void k_dup_rows(DupArgs d) {
    constexpr int SR = 3;  // super rows of a footprint of at most kSmallRows tile rows
    // per thread (entry) and super row: pairs before the row's end, super
    // tile of its first column, first column, spans of its two tile rows
    __shared__ uint32_t s_cum[SR][NT];
    __shared__ uint32_t s_first[SR][NT];
    __shared__ int32_t s_x0[SR][NT];
    __shared__ uint32_t s_sa[SR][NT];
    __shared__ uint32_t s_sb[SR][NT];
    __shared__ uint32_t s_start[NT];  // exclusive prefix of the wave's pair counts
    __shared__ uint32_t s_out[NT];    // output offset of the entry
    __shared__ uint32_t s_e[NT];      // entry id
    __shared__ uint32_t s_low[NT];    // depth bits (full-key mode)
    if (blockIdx.x == 0 && threadIdx.x == 0) pairs_clamp(d.rc, d.n_sort, d.max_pairs);
    const int64_t ne = d.rc->n_entries;
    const int lane = threadIdx.x & 63, w0 = threadIdx.x & ~63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < ne; base += gstride()) {
        const int64_t r = base + threadIdx.x;
        uint32_t n_here = 0;
        uint32_t cum[SR] = {0u, 0u, 0u}, first[SR] = {0u, 0u, 0u}, sa[SR] = {kEmptySpan, kEmptySpan, kEmptySpan},
                 sb[SR] = {kEmptySpan, kEmptySpan, kEmptySpan};
        int x0[SR] = {0, 0, 0};
        if (r < ne) {
            // two rounds of loads: (depth order, pair offset), then the
            // record's count / rows word and its spans together
            const uint32_t e = kFull ? (uint32_t)r : d.order[r];
            const uint32_t out_at = d.offs[r];
            float4* rp = d.rec + kRec * (int64_t)e;
            float4 C = make_float4(0.f, 0.f, 0.f, 0.f), D = C;
            if (d.items[r]) {  // (the entry's record is not read when it has no items)
                C = rp[2];
                D = rp[3];
            }
            const uint32_t cnt = __float_as_uint(C.w);
            if (cnt) {
                const uint32_t rows = __float_as_uint(C.y);
                const int y0 = rows & 0xffff, y1 = rows >> 16;
                if (y1 - y0 + 1 > kSmallRows) {
                    rp[3].y = __uint_as_float(out_at);  // for k_dup_big
                } else {
                    const uint32_t sp[kSmallRows] = {__float_as_uint(D.x), __float_as_uint(D.y), __float_as_uint(D.z),
                                                     __float_as_uint(D.w)};
                    const SupGeo& sg = d.sg[__float_as_uint(C.z)];
                    // super row i is Y = y0 / 2 + i: tile rows (0, 1), (2, 3)
                    // from an even y0; (-, 0), (1, 2), (3, -) from an odd one
                    const int odd = y0 & 1;
                    sa[0] = odd ? kEmptySpan : sp[0]; sb[0] = odd ? sp[0] : sp[1];
                    sa[1] = odd ? sp[1] : sp[2];      sb[1] = odd ? sp[2] : sp[3];
                    sa[2] = odd ? sp[3] : kEmptySpan; sb[2] = kEmptySpan;
                    uint32_t acc = 0;
#pragma unroll
                    for (int i = 0; i < SR; ++i) {
                        acc += sup_cols(sa[i], sb[i], x0[i]);
                        cum[i] = acc;
                        first[i] = (uint32_t)(sg.base + ((y0 >> kSupShift) + i) * sg.nsx + x0[i]);
                    }
                    n_here = acc;  // equals cnt: the spans are what was counted
                    s_out[threadIdx.x] = out_at;
                    s_e[threadIdx.x] = e;
                    s_low[threadIdx.x] = kFull ? d.dkey[e] : 0u;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            s_cum[i][threadIdx.x] = cum[i];
            s_first[i][threadIdx.x] = first[i];
            s_x0[i][threadIdx.x] = x0[i];
            s_sa[i][threadIdx.x] = sa[i];
            s_sb[i][threadIdx.x] = sb[i];
        }
        uint32_t tot;
        s_start[threadIdx.x] = wave_excl_scan(n_here, tot);
        __builtin_amdgcn_wave_barrier();  // a wave's LDS accesses complete in order
        // the wave's pairs in rank order, lane j taking pairs j, j + 64, ...:
        // consecutive lanes write consecutive slots of one entry's range
        for (uint32_t j = lane; j < tot; j += 64) {
            int lo = 0, hi = 63;  // last entry of the wave whose range starts at or before j
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_start[w0 + mid] <= j) lo = mid;
                else hi = mid - 1;
            }
            const int t = w0 + lo;
            const uint32_t k = j - s_start[t];
            int row = 0;
#pragma unroll
            for (int i = 0; i < SR - 1; ++i) row += k >= s_cum[i][t] ? 1 : 0;
            const uint32_t kk = k - (row ? s_cum[row - 1][t] : 0u);
            const uint32_t m = sup_mask(s_sa[row][t], s_sb[row][t], s_x0[row][t] + (int)kk);
            put_pair<kFull>(d, (int64_t)s_out[t] + k, s_first[row][t] + kk, s_e[t] | (m << kMaskShift), s_low[t]);
        }
        __builtin_amdgcn_wave_barrier();  // before the next step rewrites the wave's LDS
    }
}


// Dense records of the tall entries the preprocess listed per chunk of 256
// entries: chunk c's footprints at f = its offset + i (the scan's low half),
// their super rows (pairs of tile rows 2 Y, 2 Y + 1) from the chunk's
// super-row offset (the high half) on, in list order.
__global__ __launch_bounds__(NT) void k_tall_compact(const int32_t* __restrict__ list, const uint64_t* __restrict__ pack,
                                                     const uint64_t* __restrict__ off, const int32_t* n_chunks,
                                                     const float4* __restrict__ rec, TallRec* __restrict__ trec,
                                                     uint32_t* __restrict__ sroff, int64_t tall_cap,
                                                     RasterCounters* rc) {
    __shared__ uint32_t wsum[NT / 64];
    const int64_t nc = *n_chunks;
    for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {  // block-uniform
        const uint32_t n = (uint32_t)pack[c];
        const uint64_t o = off[c];
        const bool mine = threadIdx.x < n;
        int32_t x = 0;
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A, C = A;
        uint32_t nsr = 0;
        if (mine) {
            x = list[c * NT + threadIdx.x];
            const float4* rp = rec + kRec * (int64_t)x;
            A = rp[0]; B = rp[1]; C = rp[2];
            const uint32_t rows = __float_as_uint(C.y);
            nsr = ((rows >> 16) >> kSupShift) - ((rows & 0xffff) >> kSupShift) + 1;
        }
        uint32_t tot;
        const uint32_t pre = blockscan::block_excl_scan(nsr, wsum, tot);
        const int64_t f = (int64_t)(uint32_t)o + threadIdx.x;
        if (mine) {
            if (f < tall_cap) {
                const Ellipse el = make_ellipse(A.x, A.y, A.z, A.w, B.x, fmaxf(2.0f * logf(255.0f * B.y), 0.f));
                TallRec t;
                t.mx = el.mx; t.my = el.my; t.ca = el.ca; t.cb = el.cb; t.cc = el.cc; t.tau = el.tau;
                t.det = el.det; t.xmax = el.xmax; t.ymax = el.ymax; t.kr = el.kr; t.margin = el.margin;
                t.ia = el.ia; t.ic = el.ic;
                t.e = (uint32_t)x; t.rows = __float_as_uint(C.y); t.seg = __float_as_uint(C.z);
                trec[f] = t;
                sroff[f] = (uint32_t)(o >> 32) + pre;
            } else {
                atomicOr(&rc->overflow, 4);
            }
        }
    }
}

// One wave per 64 consecutive stored super rows of the tall footprints (a
// footprint's super rows are consecutive, and so are their output ranges):
// each lane loads one super row (the spans of its two tile rows, its entry
// and the items of the footprint's earlier super rows, stored by
// k_tall_spans; its columns, first super tile and output offset: the
// entry's offset, stored by k_dup_rows, plus those items) into LDS; then the
// wave writes the super rows' items, kBigGW lanes per super row, 64 /
// kBigGW at a time: lane s of a group takes items s, s + kBigGW, ... of its
// super row (consecutive lanes, consecutive slots).  No lane searches for its
// row, so the stores follow each other without LDS round trips in between.
constexpr int kBigGW = 16;
template <bool kFull>
__global__ __launch_bounds__(NT) void k_dup_big(DupArgs d) {
    constexpr int NG = 64 / kBigGW;               // super rows written at a time
    __shared__ uint4 s_row[NT / 64][64];           // (first super tile, items, output offset, entry)
    __shared__ uint4 s_sp[NT / 64][64];            // (span of tile row a, of tile row b, first column, depth bits)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int grp = lane / kBigGW, sub = lane % kBigGW;
    int64_t nr = d.rc->n_srows;
    if (nr > d.srow_cap) nr = d.srow_cap;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q0 = wave * 64; q0 < nr; q0 += nwaves * 64) {
        const int64_t q = q0 + lane;
        uint32_t np = 0, first = 0, out = 0, e = 0, low = 0, sa = kEmptySpan, sb = kEmptySpan;
        int x0 = 0;
        if (q < nr) {
            const uint4 sr = d.srow[q];
            const int y = d.srow_y[q];
            sa = sr.x;
            sb = sr.y;
            np = sup_cols(sa, sb, x0);
            if (np) {
                e = sr.z;
                const float4* rp = d.rec + kRec * (int64_t)e;
                const SupGeo& sg = d.sg[__float_as_uint(rp[2].z)];
                first = (uint32_t)(sg.base + y * sg.nsx + x0);
                out = __float_as_uint(rp[3].y) + sr.w;
                low = kFull ? d.dkey[e] : 0u;
            }
        }
        s_row[w][lane] = make_uint4(first, np, out, e);
        s_sp[w][lane] = make_uint4(sa, sb, (uint32_t)x0, low);
        __builtin_amdgcn_wave_barrier();  // a wave's LDS accesses complete in order
        const uint64_t m = __ballot(np != 0u);
        if (m) {
            const int ng = (63 - __builtin_clzll(m)) / NG + 1;  // row groups up to the last non-empty row
            uint4 nxt = s_row[w][grp], nsp = s_sp[w][grp];
            for (int g = 0; g < ng; ++g) {
                const uint4 rr = nxt, sp = nsp;
                if (g + 1 < ng) {
                    nxt = s_row[w][NG * (g + 1) + grp];
                    nsp = s_sp[w][NG * (g + 1) + grp];
                }
                for (uint32_t k = (uint32_t)sub; k < rr.y; k += kBigGW) {
                    const uint32_t mk = sup_mask(sp.x, sp.y, (int)sp.z + (int)k);
                    put_pair<kFull>(d, (int64_t)rr.z + k, rr.x + k, rr.w | (mk << kMaskShift), (uint64_t)sp.w);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();  // before the next 64 rows overwrite the arrays
    }
}

// Lanes per tall footprint in k_tall_spans (even: a super row's two tile
// rows sit in neighbouring lanes).
constexpr int kTallGW = 8;
static_assert(kTallGW % 2 == 0, "super rows pair neighbouring lanes");

// Tall footprints, kTallGW lanes each: lane s takes the footprint's tile
// rows 2 Y0 + s, 2 Y0 + s + kTallGW, ... (Y0: the footprint's first super
// row; rows outside the footprint are empty) and their exact tile spans;
// the even lane of each pair stores the pair's super row at the footprint's
// offset: (span of row 2 Y, span of row 2 Y + 1, entry, items of the
// footprint's earlier super rows) and its index Y.  The group's totals give
// the entry's tile count and its (super tile, entry) item count.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_tall_spans(SegTable tab, const TallRec* __restrict__ trec,
                                                   const uint32_t* __restrict__ sroff, RasterCounters* rc,
                                                   int64_t tall_cap, float4* __restrict__ rec, uint4* __restrict__ srow,
                                                   int32_t* __restrict__ srow_y, int64_t cap,
                                                   uint32_t* __restrict__ ntiles, uint32_t* __restrict__ nsup,
                                                   uint32_t* __restrict__ dkey) {
    int64_t n = rc->n_tall_e;
    if (n > tall_cap) n = tall_cap;
    if (gtid() == 0 && (int64_t)rc->n_srows > cap) rc->overflow |= 4;
    const int sub = (int)(threadIdx.x % kTallGW);
    const int64_t ngrp = gstride() / kTallGW;
    for (int64_t f = gtid() / kTallGW; f < n; f += ngrp) {
        const TallRec t = trec[f];
        const int64_t e = t.e;
        float4* rp = rec + kRec * e;
        const int y0 = (int)(t.rows & 0xffffu), y1 = (int)(t.rows >> 16);
        const Seg& s = tab.s[t.seg];
        Ellipse el;
        el.mx = t.mx; el.my = t.my; el.ca = t.ca; el.cb = t.cb; el.cc = t.cc; el.tau = t.tau; el.det = t.det;
        el.xmax = t.xmax; el.ymax = t.ymax; el.kr = t.kr; el.margin = t.margin; el.ia = t.ia; el.ic = t.ic;
        const int ybase = (y0 >> kSupShift) << kSupShift;  // tile row 2 Y0
        const int64_t q0 = sroff[f];
        uint32_t tiles = 0, before = 0;
        for (int b = 0; b <= y1 - ybase; b += kTallGW) {  // the group's lanes share the trip count
            const int y = ybase + b + sub;
            uint32_t sp = kEmptySpan;
            if (y >= y0 && y <= y1) {
                int lo, hi;
                row_span<false>(el, y, s.ntx, s.W, s.H, lo, hi);
                if (hi >= lo) {
                    sp = (uint32_t)lo | ((uint32_t)hi << 16);
                    tiles += (uint32_t)(hi - lo + 1);
                }
            }
            // the pair (2 Y, 2 Y + 1) of neighbouring lanes: its columns, and
            // the items of the group's earlier pairs (inclusive scan)
            const uint32_t other = (uint32_t)__shfl_xor((int)sp, 1, kTallGW);
            const bool even = !(sub & 1);
            int x0;
            const uint32_t w = even ? sup_cols(sp, other, x0) : 0u;
            uint32_t incl = w;
#pragma unroll
            for (int o = 1; o < kTallGW; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o, kTallGW);
                if (sub >= o) incl += t;
            }
            const int si = (b + sub) >> kSupShift;  // super row within the footprint
            if (even && ybase + b + sub <= y1 && q0 + si < cap) {
                srow[q0 + si] = make_uint4(sp, other, (uint32_t)e, before + incl - w);
                srow_y[q0 + si] = (ybase >> kSupShift) + si;
            }
            before += __shfl(incl, kTallGW - 1, kTallGW);
        }
#pragma unroll
        for (int o = kTallGW / 2; o > 0; o >>= 1) tiles += __shfl_xor(tiles, o, kTallGW);
        if (sub == 0) {
            rp[2].w = __uint_as_float(before);
            ntiles[e] = tiles;
            nsup[e] = before;
            if (!tiles && dkey) dkey[e] = 0u;  // (no per-entry keys when the eyes share the depth sort)
        }
    }
}



// R consecutive keys from a 16-byte aligned address, in 16-byte loads.
template <typename K, int R>
__device__ __forceinline__ void load_keys(const K* __restrict__ p, K (&k)[R]) {
    constexpr int NV = R * (int)sizeof(K) / 16;
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint4 v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = q[j];
    __builtin_memcpy(k, v, sizeof(v));
}

// Each thread scans RQ x US keys in US runs of RQ consecutive ones (plus one
// neighbour on each side of a run), so every load of a step is issued before
// any comparison.
template <typename K>
__global__ __launch_bounds__(NT) void k_ranges(const K* __restrict__ keys, const int32_t* n_sort, int shift,
                                               int32_t* __restrict__ ranges, uint32_t n_tiles) {
    // each lane takes RQ consecutive keys (a wave 64 RQ, coalesced), two such
    // steps in flight; neighbours across lanes come from the adjacent lanes,
    // the wave's two end lanes read theirs
    constexpr int RQ = sizeof(K) == 2 ? 8 : 4, US = 4;  // 16 bytes of keys per lane (32 for 64-bit keys)
    const int64_t n = *n_sort;
    const int lane = threadIdx.x & 63;
    const int64_t wave = gtid() >> 6, nwaves = gstride() >> 6;
    for (int64_t w0 = wave * (64 * RQ * US); w0 < n; w0 += nwaves * (64 * RQ * US)) {
        uint32_t t[US][RQ];
        if (w0 + 64 * RQ * US <= n) {
            // a full step: each lane's RQ keys in one load (16-byte aligned: i0 % RQ == 0)
#pragma unroll
            for (int u = 0; u < US; ++u) {
                const int64_t i0 = w0 + (int64_t)u * 64 * RQ + (int64_t)lane * RQ;
                K k[RQ];
                load_keys<K, RQ>(keys + i0, k);
#pragma unroll
                for (int q = 0; q < RQ; ++q) t[u][q] = (uint32_t)(k[q] >> shift);
            }
        } else {
#pragma unroll
            for (int u = 0; u < US; ++u) {
                const int64_t i0 = w0 + (int64_t)u * 64 * RQ + (int64_t)lane * RQ;
#pragma unroll
                for (int q = 0; q < RQ; ++q) t[u][q] = i0 + q < n ? (uint32_t)(keys[i0 + q] >> shift) : 0xffffffffu;
            }
        }
#pragma unroll
        for (int u = 0; u < US; ++u) {
            const int64_t i0 = w0 + (int64_t)u * 64 * RQ + (int64_t)lane * RQ;
            uint32_t prev = __shfl_up(t[u][RQ - 1], 1, 64), next = __shfl_down(t[u][0], 1, 64);
            if (lane == 0) prev = i0 > 0 && i0 - 1 < n ? (uint32_t)(keys[i0 - 1] >> shift) : 0xffffffffu;
            if (lane == 63) next = i0 + RQ < n ? (uint32_t)(keys[i0 + RQ] >> shift) : 0xffffffffu;
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const int64_t i = i0 + q;
                const uint32_t tq = t[u][q];
                const uint32_t pq = q == 0 ? prev : t[u][q - 1], nq = q == RQ - 1 ? next : t[u][q + 1];
                if (i < n && tq < n_tiles) {  // tq < n_tiles always holds; keeps a stray key out of bounds-safe reach
                    if (pq != tq) ranges[2 * (int64_t)tq] = (int32_t)i;
                    if (nq != tq) ranges[2 * (int64_t)tq + 1] = (int32_t)(i + 1);
                }
            }
        }
    }
}


// One wave (one block) per global tile; the block -> tile map gives each
// XCD runs of kBlendRun adjacent tiles, interleaved over the image, so
// Gaussians shared by neighbouring tiles are gathered through one L2 and the
// XCDs get equal shares of dense and sparse image regions.  Thread t owns the
// four pixels (t & 15, (t >> 4) + 4 i), i < 4, of its 16x16 tile, which share
// their column offset dx and the per-Gaussian terms that depend on it only.
// Gaussians of the tile's depth-sorted list are staged in LDS, kBlendBatch at
// a time, with the conic pre-scaled so that the exponent is base 2 and the
// log2 of the opacity folded in:
//   alpha = min(0.99, 2^(a' dx^2 + b' dx dy + c' dy^2 + log2 o)),
//   a' = -log2(e)/2 a, b' = -log2(e) b, c' = -log2(e)/2 c,
// equal to min(0.99, o exp(-q/2)) of the conic quadratic q (the hardware
// exp2 flushes results below 2^-126 to zero, far below the 1/255 cut-off).
// Per pixel: skip alpha < 1/255; stop before a Gaussian that would take
// T(1 - alpha) below 1e-4; otherwise composite.  The composite step is
// predicated (no branches); the wave stops once all its pixels are done.
static_assert(kBlendThreads == 64, "k_blend maps one wave of 64 threads onto a 16x16 tile");
template <bool kCount>
__global__ __launch_bounds__(kBlendThreads) void k_blend(SegTable tab, const int32_t* __restrict__ ranges,
                                              const uint32_t* __restrict__ vals, const float4* __restrict__ rec,
                                              uint32_t max_entries, int32_t* __restrict__ tile_eval) {
    constexpr int BB = kBlendBatch;
    __shared__ float4 sA[BB];  // mx, my, a', b'
    __shared__ float4 sB[BB];  // c', log2 o, r, g
    __shared__ float sC[BB];   // b
    constexpr float kL2e = 1.4426950408889634f;
    const int total = tab.total_tiles;
    // Blocks go to the 8 XCDs round-robin (block b to XCD b mod 8).  Each
    // run of 8 x kBlendRun blocks covers 8 runs of kBlendRun consecutive
    // tiles, one per XCD, so neighbouring tiles (which share Gaussians)
    // meet in one L2 while every XCD draws tiles from all over the image;
    // the last partial run keeps the identity map.
    const int bb = blockIdx.x, sc = bb / (8 * kBlendRun);
    const int gt = (sc + 1) * 8 * kBlendRun <= total ? sc * 8 * kBlendRun + (bb & 7) * kBlendRun + (bb % (8 * kBlendRun)) / 8
                                                      : bb;
    int si = 0;
    while (si + 1 < tab.n && gt >= tab.s[si + 1].tile_base) ++si;
    const Seg& s = tab.s[si];
    const int lt = gt - s.tile_base;
    const int tx = lt % s.ntx, ty = lt / s.ntx;
    // thread t owns the pixels (t & 15, (t >> 4) + 4 i), i < 4, of the tile
    const int px = tx * kTile + (threadIdx.x & (kTile - 1));
    const float fx = (float)px + 0.5f;
    int py[4];
    float fy[4], T[4], cr[4], cg[4], cbl[4];
    int32_t nc[4], stp[4];
    bool d[4], in[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        py[i] = ty * kTile + (threadIdx.x >> 4) + 4 * i;
        in[i] = px < s.W && py[i] < s.H;
        fy[i] = (float)py[i] + 0.5f;
        T[i] = 1.0f; cr[i] = 0.f; cg[i] = 0.f; cbl[i] = 0.f;
        nc[i] = 0; stp[i] = -1;
        d[i] = !in[i];
    }
    // the tile's list: the entries of its super tile's list whose mask has
    // the tile's bit, in list order
    const int S = s.sup_base + (ty >> kSupShift) * s.nsx + (tx >> kSupShift);
    const uint32_t bit = 1u << (kMaskShift + ((ty & 1) << 1) + (tx & 1));
    const int32_t end = ranges[2 * S + 1];
    int32_t rd = ranges[2 * S];  // next list position to read
    int32_t own = 0;             // the tile's entries staged so far
    const uint64_t below = (1ull << threadIdx.x) - 1ull;  // lanes before this one
    while (rd < end) {
        if (__all(d[0] && d[1] && d[2] && d[3])) break;
        // stage up to BB of the tile's entries: 64 list positions a step,
        // the tile's ones packed in order
        int nb = 0;
        while (nb < BB && rd < end) {
            const int32_t i = rd + (int32_t)threadIdx.x;
            const uint32_t v = i < end ? vals[i] : 0u;
            const bool mine = (v & bit) != 0u;
            const uint64_t mm = __ballot(mine);
            const int at = nb + (int)__popcll(mm & below);
            const bool take = mine && at < BB;
            const uint64_t tk = __ballot(take);
            if (take) {
                uint32_t e = v & kEntryMask;
                e = e < max_entries ? e : 0u;  // entries always are; keeps a stray id in bounds
                const float4* rp = rec + kRec * (int64_t)e;
                const float4 A = rp[0], B = rp[1];
                sA[at] = make_float4(A.x, A.y, -0.5f * kL2e * A.z, -kL2e * A.w);
                sB[at] = make_float4(-0.5f * kL2e * B.x, __log2f(B.y), B.z, B.w);
                sC[at] = rp[2].x;
            }
            nb += (int)__popcll(tk);
            // past the last position read: the whole step, or up to the last
            // entry taken when the batch filled
            rd = __popcll(mm) == __popcll(tk) ? rd + 64 : rd + 64 - (int)__builtin_clzll(tk);
        }
        // padding to the next group of 8: alpha = 2^-inf = 0 is below the
        // 1/255 cut, so these change no pixel and the unrolled loop below
        // needs no bound of its own
        for (int l = nb + (int)threadIdx.x; l < ((nb + 7) & ~7); l += kBlendThreads) {
            sA[l] = make_float4(0.f, 0.f, 0.f, 0.f);
            sB[l] = make_float4(0.f, -INFINITY, 0.f, 0.f);
            sC[l] = 0.f;
        }
        __syncthreads();
        // groups of 8: the done flags stay in scalar masks inside a group
        // and the LDS reads take immediate offsets; the padding above makes
        // a partial last group safe
        for (int k0 = 0; k0 < nb; k0 += 8) {
            if (__all(d[0] && d[1] && d[2] && d[3])) break;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = k0 + kk;
                const float4 A = sA[k];
                const float4 B = sB[k];
                const float cb = sC[k];
                const float dx = fx - A.x;
                const float u = A.w * dx;
                const float t = fmaf(A.z * dx, dx, B.y);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float e0 = fy[i] - A.y;
                    const float al = fminf(0.99f, __builtin_amdgcn_exp2f(fmaf(e0, fmaf(B.x, e0, u), t)));
                    // weight alpha T; the next transmittance T (1 - alpha) as T - alpha T
                    const float wf = al * T[i];
                    const float tn = T[i] - wf;
                    const bool uu = !d[i] && al >= kMinAlpha;
                    const bool ac = uu && tn >= kTStop;  // composite
                    const bool st = uu != ac;            // stop here (uu and not ac)
                    const float w = ac ? wf : 0.f;
                    cr[i] = fmaf(B.z, w, cr[i]); cg[i] = fmaf(B.w, w, cg[i]); cbl[i] = fmaf(cb, w, cbl[i]);
                    T[i] = ac ? tn : T[i];
                    if (kCount) {
                        nc[i] += ac ? 1 : 0;
                        stp[i] = st ? own + k : stp[i];
                    }
                    d[i] = d[i] || st;
                }
            }
        }
        own += nb;
        __syncthreads();  // the batch is read before the next one is staged
    }
    if (kCount) {
        // a pixel that never stopped visited the whole list: the loop then
        // ran to the list's end, so `own` is its length
        int32_t ne = 0, nce = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ne += in[i] ? (stp[i] >= 0 ? stp[i] + 1 : own) : 0;
            nce += nc[i];
        }
        for (int o = 32; o > 0; o >>= 1) {
            ne += __shfl_xor(ne, o);
            nce += __shfl_xor(nce, o);
        }
        if (threadIdx.x == 0) {
            tile_eval[2 * gt] = ne;
            tile_eval[2 * gt + 1] = nce;
        }
    }
    const int64_t np = (int64_t)s.W * s.H;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!in[i]) continue;
        const int64_t p = (int64_t)py[i] * s.W + px;
        s.out_rgb[p] = cr[i];
        s.out_rgb[np + p] = cg[i];
        s.out_rgb[2 * np + p] = cbl[i];
        if (s.out_T) s.out_T[p] = T[i];
        if (kCount && s.out_nc) s.out_nc[p] = nc[i];
    }
}

int bits_for(int64_t v) {
    int b = 0;
    while ((1ll << b) < v) ++b;
    return b < 1 ? 1 : b;
}

}  // namespace

void seg_camera(Seg& s, const gsc_camera& c) {
    for (int i = 0; i < 9; ++i) s.R[i] = (float)c.R[i];
    for (int i = 0; i < 3; ++i) s.pos[i] = c.pos[i];
    double tx = std::tan(0.5 * c.fovx), ty = std::tan(0.5 * c.fovy);
    s.fx = (float)(c.width / (2.0 * tx));
    s.fy = (float)(c.height / (2.0 * ty));
    s.cx = (float)(0.5 * c.width);
    s.cy = (float)(0.5 * c.height);
    s.limx = (float)(1.3 * tx);
    s.limy = (float)(1.3 * ty);
    s.znear = (float)c.znear;
    s.W = c.width;
    s.H = c.height;
    s.ntx = (c.width + kTile - 1) / kTile;
    s.nty = (c.height + kTile - 1) / kTile;
}

void seg_supers(SegTable& tab) {
    constexpr int side = 1 << kSupShift;
    int32_t b = 0;
    for (int q = 0; q < tab.n; ++q) {
        Seg& s = tab.s[q];
        s.nsx = (s.ntx + side - 1) >> kSupShift;
        s.nsy = (s.nty + side - 1) >> kSupShift;
        s.sup_base = b;
        b += s.nsx * s.nsy;
    }
    tab.total_sup = b;
}

// Paired eyes whose FP32 rotations are equal bit for bit see every point at
// view depths that differ by one constant per view (the eye offset along the
// shared optical axis), so one depth order serves both eyes up to rounding.
static bool eyes_share_rotation(const SegTable& tab) {
    if (!tab.paired || tab.n < 2 || (tab.n & 1)) return false;
    for (int q = 0; q + 1 < tab.n; q += 2)
        if (std::memcmp(tab.s[q].R, tab.s[q + 1].R, sizeof(tab.s[q].R)) != 0) return false;
    return true;
}

// Tall footprints (more than kSmallRows tile rows): dense list of the
// entries k_preprocess listed per chunk, offsets of their super rows, then
// each footprint's super rows, spans and counts.
hipError_t tall_spans(const SegTable& tab, Raster& r, hipStream_t st) {
    RasterCounters* rc = r.cnt;
    // one scan gives each chunk's first footprint (low half) and first super
    // row (high half), and the totals
    hipError_t e = scan_u64(r.pt_pack, r.pt_off, &rc->n_echunks, &rc->n_tall_e, &rc->n_srows, r.block_sums64, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tall_compact, dim3(kGridBlocks), dim3(NT), 0, st, r.pt_list, r.pt_pack, r.pt_off,
                       &rc->n_echunks, r.rec, r.trec, r.pt_sroff, r.tall_cap, rc);
    hipLaunchKernelGGL(k_tall_spans, grid_fit(k_tall_spans, r.tall_cap * kTallGW), dim3(NT), 0, st, tab, r.trec,
                       r.pt_sroff, rc, r.tall_cap, r.rec, r.srow, r.srow_y, r.srow_cap, r.ntiles, r.nsup,
                       r.shared_depth ? nullptr : r.dkey[0]);
    return hipGetLastError();
}

hipError_t raster_batch(const SegTable& tab_in, Raster& r, bool full_key_sort, bool count_work, hipStream_t st,
                        Marks* mk, hipStream_t blend_st, hipEvent_t front_done) {
    if (r.max_entries > (int64_t)kEntryMask + 1) return hipErrorInvalidValue;  // entry ids share the value with the masks
    SegTable tab = tab_in;
    seg_supers(tab);
    RasterCounters* rc = r.cnt;
    mark(mk, 3, st);
    PreArgs pa;
    pa.tab = tab; pa.rc = rc; pa.rec = r.rec; pa.ntiles = r.ntiles; pa.nsup = r.nsup; pa.dkey = r.dkey[0];
    pa.dval = r.dval[0];
    pa.tall_list = r.pt_list; pa.tall_pack = r.pt_pack; pa.ranges = r.ranges; pa.n_ranges = 2 * (int64_t)tab.total_sup;
    pa.max_entries = r.max_entries;
    r.shared_depth = !full_key_sort && eyes_share_rotation(tab);
    pa.shared_depth = r.shared_depth ? 1 : 0;
    hipLaunchKernelGGL(k_preprocess, grid_fit(k_preprocess, r.max_entries), dim3(NT), 0, st, pa);
    mark(mk, 4, st);
    hipError_t e0 = tall_spans(tab, r, st);
    if (e0 != hipSuccess) return e0;
    mark(mk, 5, st);
    const int tile_bits = bits_for(tab.total_sup);  // the sort's key: the global super-tile id
    DupArgs da;
    for (int q = 0; q < kMaxSeg; ++q) da.sg[q] = SupGeo{q < tab.n ? tab.s[q].sup_base : 0, q < tab.n ? tab.s[q].nsx : 0};
    da.rc = rc; da.rec = r.rec; da.max_pairs = r.max_pairs; da.dkey = r.dkey[0];
    da.srow = r.srow; da.srow_y = r.srow_y; da.srow_cap = r.srow_cap; da.n_sort = r.n_sort;
    hipError_t e;
    if (!full_key_sort) {
        // low 32 key bits (depth) first, per Gaussian
        int which = 0;
        // the last pass also lays the tile counts out in depth order (scnt);
        // with a shared sort it sorts the Gaussians and lays out both eyes'
        // entries of each at neighbouring ranks
        e = radix_sort_u32(r.dkey, r.dval, r.shared_depth ? &rc->n_gpairs : &rc->n_entries, 0, 0, 32, r.hist,
                           r.block_sums, &which, st, r.nsup, r.scnt, r.shared_depth);
        if (e != hipSuccess) return e;
        mark(mk, 6, st);
        e = scan_u32(r.scnt, r.offs, &rc->n_entries, 0, &rc->n_pairs, r.block_sums, st);
        if (e != hipSuccess) return e;
        mark(mk, 7, st);
        // keys in 16 bits when the batch's global super-tile ids fit
        const bool k16 = tab.total_sup <= 65536;
        uint16_t* pk16[2] = {reinterpret_cast<uint16_t*>(r.pkey[0]), reinterpret_cast<uint16_t*>(r.pkey[1])};
        da.order = r.dval[which]; da.offs = r.offs; da.items = r.scnt; da.key64 = nullptr; da.val = r.pval[0];
        da.key32 = k16 ? nullptr : r.pkey[0];
        da.key16 = k16 ? pk16[0] : nullptr;
        hipLaunchKernelGGL(k_dup_rows<false>, grid_fit(k_dup_rows<false>, r.max_entries), dim3(NT), 0, st, da);
        mark(mk, 8, st);
        mark(mk, 9, st);  // (no kernel in the tall-list stage: k_dup_big reads the stored super rows)
        hipLaunchKernelGGL(k_dup_big<false>, grid_fit(k_dup_big<false>, r.srow_cap), dim3(NT), 0, st, da);
        mark(mk, 10, st);
        // then the tile bits, on the pairs (stable: depth order kept per tile)
        int pw = 0;
        e = k16 ? radix_sort_u16(pk16, r.pval, r.n_sort, 0, 0, tile_bits, r.hist, r.block_sums, &pw, st)
                : radix_sort_u32(r.pkey, r.pval, r.n_sort, 0, 0, tile_bits, r.hist, r.block_sums, &pw, st);
        if (e != hipSuccess) return e;
        mark(mk, 11, st);
        r.sorted_buf = pw;
        r.key16 = k16;
        if (k16)
            hipLaunchKernelGGL(k_ranges<uint16_t>, grid_fit(k_ranges<uint16_t>, r.max_pairs / 8 + 1), dim3(NT), 0, st,
                               pk16[pw], r.n_sort, 0, r.ranges, (uint32_t)tab.total_sup);
        else
            hipLaunchKernelGGL(k_ranges<uint32_t>, grid_fit(k_ranges<uint32_t>, r.max_pairs / 8 + 1), dim3(NT), 0, st,
                               r.pkey[pw], r.n_sort, 0, r.ranges, (uint32_t)tab.total_sup);
    } else {
        mark(mk, 6, st);  // no per-Gaussian depth pass in this mode
        e = scan_u32(r.nsup, r.offs, &rc->n_entries, 0, &rc->n_pairs, r.block_sums, st);
        if (e != hipSuccess) return e;
        mark(mk, 7, st);
        da.order = nullptr; da.offs = r.offs; da.items = r.nsup; da.key32 = nullptr; da.key16 = nullptr; da.key64 = r.pkey64[0];
        da.val = r.pval[0];
        r.key16 = false;
        hipLaunchKernelGGL(k_dup_rows<true>, grid_fit(k_dup_rows<true>, r.max_entries), dim3(NT), 0, st, da);
        mark(mk, 8, st);
        mark(mk, 9, st);
        hipLaunchKernelGGL(k_dup_big<true>, grid_fit(k_dup_big<true>, r.srow_cap), dim3(NT), 0, st, da);
        mark(mk, 10, st);
        int pw = 0;
        e = radix_sort_u64(r.pkey64, r.pval, r.n_sort, 0, 0, 32 + tile_bits, r.hist, r.block_sums, &pw, st);
        if (e != hipSuccess) return e;
        mark(mk, 11, st);
        r.sorted_buf = pw;
        hipLaunchKernelGGL(k_ranges<uint64_t>, grid_fit(k_ranges<uint64_t>, r.max_pairs / 8 + 1), dim3(NT), 0, st, r.pkey64[pw], r.n_sort,
                           32, r.ranges, (uint32_t)tab.total_sup);
    }
    r.order = nullptr;
    hipStream_t bs = st;
    if (blend_st && blend_st != st) {
        e = hipEventRecord(front_done, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(blend_st, front_done, 0);
        if (e != hipSuccess) return e;
        bs = blend_st;
    }
    mark(mk, 12, bs);
    if (count_work)
        hipLaunchKernelGGL(k_blend<true>, dim3((unsigned)tab.total_tiles), dim3(kBlendThreads), 0, bs, tab, r.ranges,
                           r.pval[r.sorted_buf], r.rec, (uint32_t)r.max_entries, r.tile_eval);
    else
        hipLaunchKernelGGL(k_blend<false>, dim3((unsigned)tab.total_tiles), dim3(kBlendThreads), 0, bs, tab, r.ranges,
                           r.pval[r.sorted_buf], r.rec, (uint32_t)r.max_entries, r.tile_eval);
    mark(mk, 13, bs);
    return hipGetLastError();
}

}  // namespace gsc
