// Raster stage (Section 3.1 splatting + Section 6 RasterizeGaussians) for a
// batch of images ("segments": one per (viewer, eye)), all in one set of
// launches:
//   k_entry_bases      segment -> first entry (counts stay on the device)
//   k_preprocess       EWA projection, conic, opacity-aware extent, exact
//                      tile count, depth key                (per entry)
//   depth radix pass   stable sort of entries by float32 depth (the low 32
//                      bits of the (tile | depth) key, applied per Gaussian
//                      before duplication)
//   scan + k_duplicate one (global tile id, entry) pair per covered tile,
//                      emitted in depth order
//   tile radix pass    stable sort of pairs by global tile id (the high bits)
//   k_ranges           [start, end) of every tile's run
//   k_blend            front-to-back compositing, one block per tile,
//                      LDS-staged Gaussian batches, block-wide early exit
// With full_key_sort the pairs carry the whole 64-bit (tile << 32 | depth)
// key and are sorted after duplication instead; the order is the same.
#include <cmath>

#include "gsc_common.h"

namespace gsc {

namespace {

constexpr int NT = 256;
constexpr float kMinAlpha = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;

__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

inline dim3 grid_for(int64_t n) {
    int64_t b = (n + NT - 1) / NT;
    if (b < 1) b = 1;
    if (b > kGridBlocks) b = kGridBlocks;
    return dim3((unsigned)b);
}

__device__ __forceinline__ int seg_of_entry(const RasterCounters* rc, int nseg, int64_t e) {
    int s = 0;
    while (s + 1 < nseg && e >= rc->entry_base[s + 1]) ++s;
    return s;
}

__global__ void k_entry_bases(SegTable tab, RasterCounters* rc, int64_t max_entries) {
    int32_t acc = 0;
    for (int s = 0; s < tab.n; ++s) {
        rc->entry_base[s] = acc;
        int32_t n = tab.s[s].nG ? *tab.s[s].nG : tab.s[s].nG_host;
        acc += n;
        rc->seg_pairs[s] = 0;
    }
    rc->entry_base[tab.n] = acc;
    rc->overflow = 0;
    if (acc > max_entries) {
        rc->overflow |= 2;
        acc = (int32_t)max_entries;
    }
    rc->n_entries = acc;
}

// Minimum of q(d) = a dx^2 + 2 b dx dy + c dy^2 over the closed rectangle
// [x0,x1] x [y0,y1] of offsets d (q convex: 0 inside, else on an edge).
// Contraction is off so that the count and emit passes agree exactly.
__device__ __forceinline__ float rect_min_q(float a, float b, float c, float x0, float x1, float y0, float y1) {
#pragma clang fp contract(off)
    if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return 0.f;
    float best = INFINITY;
    float fx[2] = {x0, x1}, fy[2] = {y0, y1};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        float dx = fx[i];
        float dy = fminf(fmaxf(-b * dx / c, y0), y1);
        best = fminf(best, a * dx * dx + 2.f * b * dx * dy + c * dy * dy);
        float ey = fy[i];
        float ex = fminf(fmaxf(-b * ey / a, x0), x1);
        best = fminf(best, a * ex * ex + 2.f * b * ex * ey + c * ey * ey);
    }
    return best;
}

// Does the footprint {q <= tau} of a Gaussian centred at (mx, my) reach the
// pixel-centre rectangle of tile (tx, ty)?
__device__ __forceinline__ bool tile_hit(float mx, float my, float ca, float cb, float cc, float tau, int tx, int ty,
                                         int W, int H) {
#pragma clang fp contract(off)
    float x0 = (float)(kTile * tx) + 0.5f, y0 = (float)(kTile * ty) + 0.5f;
    float x1 = (float)min(kTile * tx + kTile - 1, W - 1) + 0.5f;
    float y1 = (float)min(kTile * ty + kTile - 1, H - 1) + 0.5f;
    return rect_min_q(ca, cb, cc, x0 - mx, x1 - mx, y0 - my, y1 - my) <= tau;
}

struct PreArgs {
    SegTable tab;
    RasterCounters* rc;
    float4* recA;
    float4* recB;
    float* recC;
    uint32_t* ntiles;
    uint2* rect;
    uint32_t* dkey;
    uint32_t* dval;
};

__global__ __launch_bounds__(NT) void k_preprocess(PreArgs p) {
    const int64_t ne = p.rc->n_entries;
    for (int64_t e = gtid(); e < ne; e += gstride()) {
        int si = seg_of_entry(p.rc, p.tab.n, e);
        const Seg& s = p.tab.s[si];
        int64_t g = e - p.rc->entry_base[si];
        int64_t src = s.G ? (int64_t)s.G[g] : g;
        float4 l0 = s.L0[src], l1 = s.L1[src], l2 = s.L2[src];
        float lb = s.L3[src];
        uint32_t count = 0;
        float depth = 0.f;
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = make_float4(0.f, 0.f, 0.f, 0.f);
        uint2 rc = make_uint2(0u, 0u);
        float vx = l0.x - s.pos[0], vy = l0.y - s.pos[1], vz = l0.z - s.pos[2];
        float tx = s.R[0] * vx + s.R[1] * vy + s.R[2] * vz;
        float ty = s.R[3] * vx + s.R[4] * vy + s.R[5] * vz;
        float tz = s.R[6] * vx + s.R[7] * vy + s.R[8] * vz;
        float alpha = l0.w;
        if (tz > s.znear && alpha >= kMinAlpha) {
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
                float tau = 2.0f * logf(255.0f * alpha);
                tau = fmaxf(tau, 0.f);
                float cdet = ca * cc - cb * cb;
                float sxx = cc / cdet, syy = ca / cdet;
                float ex = sqrtf(tau * sxx) + 1.0f, ey = sqrtf(tau * syy) + 1.0f;
                float fx0 = floorf((mx - ex - 0.5f) * (1.0f / kTile)), fx1 = floorf((mx + ex - 0.5f) * (1.0f / kTile));
                float fy0 = floorf((my - ey - 0.5f) * (1.0f / kTile)), fy1 = floorf((my + ey - 0.5f) * (1.0f / kTile));
                int x0 = (int)fminf(fmaxf(fx0, 0.f), (float)(s.ntx - 1)), x1 = (int)fminf(fmaxf(fx1, -1.f), (float)(s.ntx - 1));
                int y0 = (int)fminf(fmaxf(fy0, 0.f), (float)(s.nty - 1)), y1 = (int)fminf(fmaxf(fy1, -1.f), (float)(s.nty - 1));
                if (fx0 > (float)(s.ntx - 1) || fy0 > (float)(s.nty - 1)) x1 = -1;
                if (x0 <= x1 && y0 <= y1) {
                    for (int yy = y0; yy <= y1; ++yy)
                        for (int xx = x0; xx <= x1; ++xx)
                            count += tile_hit(mx, my, ca, cb, cc, tau, xx, yy, s.W, s.H) ? 1u : 0u;
                    rc = make_uint2((uint32_t)x0 | ((uint32_t)x1 << 16), (uint32_t)y0 | ((uint32_t)y1 << 16));
                }
            }
        }
        p.recA[e] = A;
        p.recB[e] = B;
        p.recC[e] = lb;
        p.rect[e] = rc;
        p.ntiles[e] = count;
        p.dkey[e] = count ? __float_as_uint(depth) : 0u;
        p.dval[e] = (uint32_t)e;
    }
}

// counts in depth order for the offset scan
__global__ __launch_bounds__(NT) void k_gather_counts(const uint32_t* __restrict__ order, const uint32_t* __restrict__ ntiles,
                                                      const RasterCounters* rc, uint32_t* __restrict__ out) {
    const int64_t ne = rc->n_entries;
    for (int64_t r = gtid(); r < ne; r += gstride()) out[r] = ntiles[order[r]];
}

struct DupArgs {
    SegTable tab;
    RasterCounters* rc;
    const uint32_t* order;   // depth-sorted entry ids (nullptr = entry order)
    const uint32_t* offs;    // pair offset per rank
    const uint32_t* ntiles;
    const uint2* rect;
    const float4* recA;
    const float4* recB;
    uint32_t* key32;         // global tile id (depth-presorted mode)
    uint64_t* key64;         // (global tile << 32 | depth bits) (full-key mode)
    uint32_t* val;
    int64_t max_pairs;
};

__global__ __launch_bounds__(NT) void k_duplicate(DupArgs d) {
    const int64_t ne = d.rc->n_entries;
    for (int64_t r = gtid(); r < ne; r += gstride()) {
        uint32_t e = d.order[r];
        uint32_t cnt = d.ntiles[e];
        if (!cnt) continue;
        int si = seg_of_entry(d.rc, d.tab.n, e);
        const Seg& s = d.tab.s[si];
        float4 A = d.recA[e], B = d.recB[e];
        float tau = fmaxf(2.0f * logf(255.0f * B.y), 0.f);
        uint2 rc = d.rect[e];
        int x0 = rc.x & 0xffff, x1 = rc.x >> 16, y0 = rc.y & 0xffff, y1 = rc.y >> 16;
        int64_t o = d.offs[r];
        uint32_t w = 0;
        for (int yy = y0; yy <= y1 && w < cnt; ++yy)
            for (int xx = x0; xx <= x1 && w < cnt; ++xx) {
                if (!tile_hit(A.x, A.y, A.z, A.w, B.x, tau, xx, yy, s.W, s.H)) continue;
                int64_t q = o + w;
                ++w;
                if (q >= d.max_pairs) continue;
                d.key32[q] = (uint32_t)(s.tile_base + yy * s.ntx + xx);
                d.val[q] = e;
            }
    }
}

__global__ __launch_bounds__(NT) void k_duplicate64(DupArgs d, const uint32_t* __restrict__ dkey) {
    const int64_t ne = d.rc->n_entries;
    for (int64_t e = gtid(); e < ne; e += gstride()) {
        uint32_t cnt = d.ntiles[e];
        if (!cnt) continue;
        int si = seg_of_entry(d.rc, d.tab.n, e);
        const Seg& s = d.tab.s[si];
        float4 A = d.recA[e], B = d.recB[e];
        float tau = fmaxf(2.0f * logf(255.0f * B.y), 0.f);
        uint2 rc = d.rect[e];
        int x0 = rc.x & 0xffff, x1 = rc.x >> 16, y0 = rc.y & 0xffff, y1 = rc.y >> 16;
        int64_t o = d.offs[e];
        uint32_t w = 0;
        uint64_t low = dkey[e];
        for (int yy = y0; yy <= y1 && w < cnt; ++yy)
            for (int xx = x0; xx <= x1 && w < cnt; ++xx) {
                if (!tile_hit(A.x, A.y, A.z, A.w, B.x, tau, xx, yy, s.W, s.H)) continue;
                int64_t q = o + w;
                ++w;
                if (q >= d.max_pairs) continue;
                uint64_t gt = (uint64_t)(s.tile_base + yy * s.ntx + xx);
                d.key64[q] = (gt << 32) | low;
                d.val[q] = (uint32_t)e;
            }
    }
}

__global__ void k_pairs_clamp(RasterCounters* rc, int32_t* n_sort, int64_t max_pairs) {
    int32_t n = rc->n_pairs;
    if ((int64_t)n > max_pairs) {
        rc->overflow |= 1;
        n = (int32_t)max_pairs;
    }
    *n_sort = n;
}

__global__ __launch_bounds__(NT) void k_fill_ranges(int32_t* __restrict__ ranges, int64_t n2) {
    for (int64_t i = gtid(); i < n2; i += gstride()) ranges[i] = 0;
}

template <typename K>
__global__ __launch_bounds__(NT) void k_ranges(const K* __restrict__ keys, const int32_t* n_sort, int shift,
                                               int32_t* __restrict__ ranges) {
    const int64_t n = *n_sort;
    for (int64_t i = gtid(); i < n; i += gstride()) {
        uint32_t t = (uint32_t)(keys[i] >> shift);
        if (i == 0 || (uint32_t)(keys[i - 1] >> shift) != t) ranges[2 * (int64_t)t] = (int32_t)i;
        if (i == n - 1 || (uint32_t)(keys[i + 1] >> shift) != t) ranges[2 * (int64_t)t + 1] = (int32_t)(i + 1);
    }
}

// Per-segment pair counts (stats): one block per segment sums its tiles' runs.
__global__ __launch_bounds__(NT) void k_seg_pairs(const int32_t* __restrict__ ranges, SegTable tab, RasterCounters* rc) {
    __shared__ int32_t part[NT];
    const Seg& g = tab.s[blockIdx.x];
    int64_t t0 = g.tile_base, t1 = g.tile_base + (int64_t)g.ntx * g.nty;
    int32_t acc = 0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += NT) acc += ranges[2 * t + 1] - ranges[2 * t];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) rc->seg_pairs[blockIdx.x] = part[0];
}

// One block per global tile; block -> tile mapping keeps runs of adjacent
// tiles on one XCD (blocks are dealt round-robin over the 8 XCDs) so that
// Gaussians shared by neighbouring tiles are gathered through one L2.
__global__ __launch_bounds__(kBlendThreads) void k_blend(SegTable tab, const int32_t* __restrict__ ranges,
                                                          const uint32_t* __restrict__ vals,
                                                          const float4* __restrict__ recA,
                                                          const float4* __restrict__ recB,
                                                          const float* __restrict__ recC) {
    __shared__ float4 sA[kBlendThreads];
    __shared__ float4 sB[kBlendThreads];
    __shared__ float sC[kBlendThreads];
    const int total = tab.total_tiles;
    const int q8 = total >> 3, r8 = total & 7;
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int gt = xcd * q8 + min(xcd, r8) + j;
    int si = 0;
    while (si + 1 < tab.n && gt >= tab.s[si + 1].tile_base) ++si;
    const Seg& s = tab.s[si];
    const int lt = gt - s.tile_base;
    const int tx = lt % s.ntx, ty = lt / s.ntx;
    const int px = tx * kTile + (threadIdx.x & (kTile - 1));
    const int py = ty * kTile + (threadIdx.x / kTile);
    const bool inside = px < s.W && py < s.H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const int32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
    float T = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    int32_t nc = 0;
    bool done = !inside;
    for (int32_t base = start; base < end; base += kBlendThreads) {
        if (__syncthreads_count(done) == kBlendThreads) break;
        int32_t i = base + (int32_t)threadIdx.x;
        if (i < end) {
            uint32_t e = vals[i];
            sA[threadIdx.x] = recA[e];
            sB[threadIdx.x] = recB[e];
            sC[threadIdx.x] = recC[e];
        }
        __syncthreads();
        const int nb = min(kBlendThreads, end - base);
        if (!done) {
            for (int k = 0; k < nb; ++k) {
                float4 A = sA[k];
                float4 B = sB[k];
                float dx = fx - A.x, dy = fy - A.y;
                float q = A.z * dx * dx + 2.0f * A.w * dx * dy + B.x * dy * dy;
                float al = fminf(0.99f, B.y * __expf(-0.5f * q));
                if (al < kMinAlpha) continue;
                float tn = T * (1.0f - al);
                if (tn < kTStop) {
                    done = true;
                    break;
                }
                float w = al * T;
                c0 += B.z * w;
                c1 += B.w * w;
                c2 += sC[k] * w;
                T = tn;
                ++nc;
            }
        }
    }
    if (inside) {
        const int64_t p = (int64_t)py * s.W + px, np = (int64_t)s.W * s.H;
        s.out_rgb[p] = c0;
        s.out_rgb[np + p] = c1;
        s.out_rgb[2 * np + p] = c2;
        if (s.out_T) s.out_T[p] = T;
        if (s.out_nc) s.out_nc[p] = nc;
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
    for (int i = 0; i < 3; ++i) s.pos[i] = (float)c.pos[i];
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

hipError_t raster_batch(const SegTable& tab, Raster& r, bool full_key_sort, hipStream_t st) {
    RasterCounters* rc = r.cnt;
    hipLaunchKernelGGL(k_entry_bases, dim3(1), dim3(1), 0, st, tab, rc, r.max_entries);
    PreArgs pa;
    pa.tab = tab; pa.rc = rc; pa.recA = r.recA; pa.recB = r.recB; pa.recC = r.recC; pa.ntiles = r.ntiles;
    pa.rect = r.rect; pa.dkey = r.dkey[0]; pa.dval = r.dval[0];
    hipLaunchKernelGGL(k_preprocess, grid_for(r.max_entries), dim3(NT), 0, st, pa);
    const int tile_bits = bits_for(tab.total_tiles);
    DupArgs da;
    da.tab = tab; da.rc = rc; da.ntiles = r.ntiles; da.rect = r.rect; da.recA = r.recA; da.recB = r.recB;
    da.max_pairs = r.max_pairs;
    hipError_t e;
    if (!full_key_sort) {
        int which = 0;
        e = radix_sort_u32(r.dkey, r.dval, &rc->n_entries, 0, 0, 32, r.hist, r.block_sums, &which, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_gather_counts, grid_for(r.max_entries), dim3(NT), 0, st, r.dval[which], r.ntiles, rc,
                           r.dkey[which ^ 1]);
        e = scan_u32(r.dkey[which ^ 1], r.offs, &rc->n_entries, 0, &rc->n_pairs, r.block_sums, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_pairs_clamp, dim3(1), dim3(1), 0, st, rc, r.n_sort, r.max_pairs);
        da.order = r.dval[which]; da.offs = r.offs; da.key32 = r.pkey[0]; da.key64 = nullptr; da.val = r.pval[0];
        hipLaunchKernelGGL(k_duplicate, grid_for(r.max_entries), dim3(NT), 0, st, da);
        int pw = 0;
        e = radix_sort_u32(r.pkey, r.pval, r.n_sort, 0, 0, tile_bits, r.hist, r.block_sums, &pw, st);
        if (e != hipSuccess) return e;
        r.sorted_buf = pw;
        hipLaunchKernelGGL(k_fill_ranges, grid_for(2 * r.max_tiles), dim3(NT), 0, st, r.ranges, 2 * (int64_t)tab.total_tiles);
        hipLaunchKernelGGL(k_ranges<uint32_t>, grid_for(r.max_pairs), dim3(NT), 0, st, r.pkey[pw], r.n_sort, 0,
                           r.ranges);
    } else {
        e = scan_u32(r.ntiles, r.offs, &rc->n_entries, 0, &rc->n_pairs, r.block_sums, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_pairs_clamp, dim3(1), dim3(1), 0, st, rc, r.n_sort, r.max_pairs);
        da.order = nullptr; da.offs = r.offs; da.key32 = nullptr; da.key64 = r.pkey64[0]; da.val = r.pval[0];
        hipLaunchKernelGGL(k_duplicate64, grid_for(r.max_entries), dim3(NT), 0, st, da, r.dkey[0]);
        int pw = 0;
        e = radix_sort_u64(r.pkey64, r.pval, r.n_sort, 0, 0, 32 + tile_bits, r.hist, r.block_sums, &pw, st);
        if (e != hipSuccess) return e;
        r.sorted_buf = pw;
        hipLaunchKernelGGL(k_fill_ranges, grid_for(2 * r.max_tiles), dim3(NT), 0, st, r.ranges, 2 * (int64_t)tab.total_tiles);
        hipLaunchKernelGGL(k_ranges<uint64_t>, grid_for(r.max_pairs), dim3(NT), 0, st, r.pkey64[pw], r.n_sort, 32,
                           r.ranges);
    }
    hipLaunchKernelGGL(k_seg_pairs, dim3((unsigned)tab.n), dim3(NT), 0, st, r.ranges, tab, rc);
    hipLaunchKernelGGL(k_blend, dim3((unsigned)tab.total_tiles), dim3(kBlendThreads), 0, st, tab, r.ranges,
                       r.pval[r.sorted_buf], r.recA, r.recB, r.recC);
    return hipGetLastError();
}

}  // namespace gsc
