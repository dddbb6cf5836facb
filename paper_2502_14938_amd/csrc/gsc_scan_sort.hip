// Device-wide primitives: exclusive scan and stable LSD radix sort.
//
// Both use a fixed grid whose blocks own contiguous chunks of the input and
// read the element count from device memory, so a frame never needs a host
// round trip to size a launch.  Wave64 throughout: wave scans use
// __shfl_up over 64 lanes, digit ranking uses 64-bit ballots.
#include "gsc_blockscan.h"
#include "gsc_common.h"

namespace gsc {

namespace {

constexpr int NT = 256;        // threads per block (4 waves)
constexpr int SCAN_TILE = 1024;  // elements per scan step (4 per thread)
constexpr int SORT_IPT_U32 = 8;
constexpr int SORT_IPT_U16 = 16;
// Elements per thread per sort step, by key width: the depth sort (32-bit
// keys, one per Gaussian) is small enough that 16 per thread would leave
// most of the chip idle, so its tiles are half as long.
template <typename K>
constexpr int sort_ipt() { return sizeof(K) == 4 ? SORT_IPT_U32 : sizeof(K) == 2 ? SORT_IPT_U16 : 16; }
template <typename K>
constexpr int sort_tile() { return NT * sort_ipt<K>(); }

using blockscan::block_carry;
using blockscan::block_excl_scan;
using blockscan::block_sum;
using blockscan::chunk_of;
using blockscan::count_of;
static_assert(NT == blockscan::kThreads && SCAN_TILE == blockscan::kTile, "scan block shape");

// ------------------------------------------------------------------ scan

__global__ __launch_bounds__(NT) void k_scan_reduce(const uint32_t* __restrict__ in, const int32_t* n_dev,
                                                    int64_t n_host, uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t wsum[NT / 64];
    int64_t b0, b1;
    chunk_of(count_of(n_dev, n_host), SCAN_TILE, b0, b1);
    uint32_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += NT) s += in[i];
    uint32_t t = block_sum(s, wsum);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = t;
}

// Each block takes its carry as the sum of the preceding blocks' sums (a
// block reduction, no separate pass over the block sums); the last block
// writes the total.
__global__ __launch_bounds__(NT) void k_scan_down(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                  const int32_t* n_dev, int64_t n_host,
                                                  const uint32_t* __restrict__ block_sums, int32_t* total) {
    __shared__ uint32_t wsum[NT / 64];
    uint32_t carry = block_carry(block_sums, wsum, total);
    int64_t b0, b1;
    chunk_of(count_of(n_dev, n_host), SCAN_TILE, b0, b1);
    for (int64_t base = b0; base < b1; base += SCAN_TILE) {
        uint32_t v[4], s = 0;
        int64_t i0 = base + threadIdx.x * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v[r] = i0 + r < b1 ? in[i0 + r] : 0u;
            s += v[r];
        }
        uint32_t tot;
        uint32_t e = carry + block_excl_scan(s, wsum, tot);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (i0 + r < b1) out[i0 + r] = e;
            e += v[r];
        }
        carry += tot;
    }
}

// 64-bit form: each value packs two 32-bit counts (low, high) that scan
// independently; the totals go to total_lo and total_hi.
__global__ __launch_bounds__(NT) void k_scan_reduce64(const uint64_t* __restrict__ in, const int32_t* n_dev,
                                                      uint64_t* __restrict__ block_sums) {
    __shared__ uint64_t wsum[NT / 64];
    int64_t b0, b1;
    chunk_of(count_of(n_dev, 0), SCAN_TILE, b0, b1);
    uint64_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += NT) s += in[i];
    uint64_t t = block_sum<uint64_t>(s, wsum);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = t;
}

__global__ __launch_bounds__(NT) void k_scan_down64(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                    const int32_t* n_dev, const uint64_t* __restrict__ block_sums,
                                                    int32_t* total_lo, int32_t* total_hi) {
    __shared__ uint64_t wsum[NT / 64];
    uint64_t carry = block_carry<uint64_t>(block_sums, wsum);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const uint64_t t = carry + block_sums[blockIdx.x];
        *total_lo = (int32_t)(uint32_t)t;
        *total_hi = (int32_t)(uint32_t)(t >> 32);
    }
    int64_t b0, b1;
    chunk_of(count_of(n_dev, 0), SCAN_TILE, b0, b1);
    for (int64_t base = b0; base < b1; base += SCAN_TILE) {
        uint64_t v[4], s = 0;
        int64_t i0 = base + threadIdx.x * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v[r] = i0 + r < b1 ? in[i0 + r] : 0ull;
            s += v[r];
        }
        uint64_t tot;
        uint64_t e = carry + block_excl_scan<uint64_t>(s, wsum, tot);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (i0 + r < b1) out[i0 + r] = e;
            e += v[r];
        }
        carry += tot;
    }
}

// Compaction form of the down-sweep: flags in `in` (0 or 1), and
// ids[prefix] = i for every flagged i (ascending).
__global__ __launch_bounds__(NT) void k_scan_compact(const uint32_t* __restrict__ in, int32_t* __restrict__ ids,
                                                     const int32_t* n_dev, int64_t n_host,
                                                     const uint32_t* __restrict__ block_sums, int32_t* total) {
    __shared__ uint32_t wsum[NT / 64];
    uint32_t carry = block_carry(block_sums, wsum, total);
    int64_t b0, b1;
    chunk_of(count_of(n_dev, n_host), SCAN_TILE, b0, b1);
    for (int64_t base = b0; base < b1; base += SCAN_TILE) {
        uint32_t v[4], s = 0;
        int64_t i0 = base + threadIdx.x * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v[r] = i0 + r < b1 ? in[i0 + r] : 0u;
            s += v[r];
        }
        uint32_t tot;
        uint32_t e = carry + block_excl_scan(s, wsum, tot);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (v[r]) ids[e] = (int32_t)(i0 + r);
            e += v[r];
        }
        carry += tot;
    }
}

// ------------------------------------------------------------ radix sort

template <typename K>
__device__ __forceinline__ uint32_t digit(K key, int shift, uint32_t mask) {
    return (uint32_t)(key >> shift) & mask;
}

// Lanes of the wave holding the same BITS-bit digit (among the valid ones).
// A lane differs from this one where some digit bit's ballot differs from
// this lane's own bit, so the complement of OR over bits of (ballot XOR own
// bit replicated to 32 bits), in two 32-bit halves, is the peer set.
template <int BITS>
__device__ __forceinline__ uint64_t peers_of(uint32_t d, bool valid) {
    const uint64_t vb = __ballot(valid);
    uint32_t lo = ~(uint32_t)vb, hi = ~(uint32_t)(vb >> 32);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint32_t t = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);  // bit b: 0 or all ones
        const uint64_t bb = __ballot(t != 0u);
        lo |= (uint32_t)bb ^ t;
        hi |= (uint32_t)(bb >> 32) ^ t;
    }
    return ~(((uint64_t)hi << 32) | (uint64_t)lo);
}

// IPT consecutive keys starting at a 16-byte aligned element.
template <typename K, int IPT>
__device__ __forceinline__ void load_run(const K* __restrict__ p, K (&k)[IPT]) {
    static_assert(IPT * sizeof(K) % 16 == 0, "whole 16-byte loads");
    constexpr int NV = IPT * (int)sizeof(K) / 16;
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint4 v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = q[j];
    __builtin_memcpy(k, v, sizeof(v));
}

// Digit counts of the block's chunk.  Each thread takes SORT_IPT
// consecutive keys and adds each run of equal digits in one update of its
// wave's LDS counters, so keys that come in runs (the tile ids of one
// footprint row, the high digits of nearby depths) cost one update per run.
template <typename K>
__global__ __launch_bounds__(NT) void k_radix_hist(const K* __restrict__ keys, const int32_t* n_dev, int64_t n_host,
                                                   int shift, int bits, uint32_t* __restrict__ hist) {
    constexpr int SORT_IPT = sort_ipt<K>(), SORT_TILE = sort_tile<K>();
    __shared__ uint32_t h[4][256];
    const int w = threadIdx.x >> 6;
    const uint32_t nbins = 1u << bits, mask = nbins - 1u;
    for (int i = threadIdx.x; i < 4 * 256; i += NT) (&h[0][0])[i] = 0u;
    __syncthreads();
    int64_t b0, b1;
    chunk_of(count_of(n_dev, n_host), SORT_TILE, b0, b1);
    for (int64_t base = b0; base < b1; base += SORT_TILE) {
        const int64_t i0 = base + (int64_t)threadIdx.x * SORT_IPT;
        const int m = i0 >= b1 ? 0 : (b1 - i0 < SORT_IPT ? (int)(b1 - i0) : SORT_IPT);
        K k[SORT_IPT];
        if (m == SORT_IPT) {
            load_run(keys + i0, k);
        } else {
#pragma unroll
            for (int r = 0; r < SORT_IPT; ++r) k[r] = r < m ? keys[i0 + r] : (K)0;
        }
        if (m == 0) continue;
        uint32_t cur = digit(k[0], shift, mask), run = 1u;
#pragma unroll
        for (int r = 1; r < SORT_IPT; ++r) {
            if (r < m) {
                const uint32_t d = digit(k[r], shift, mask);
                if (d != cur) {
                    atomicAdd(&h[w][cur], run);
                    cur = d;
                    run = 0u;
                }
                ++run;
            }
        }
        atomicAdd(&h[w][cur], run);
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < nbins; q += NT)
        hist[(int64_t)q * gridDim.x + blockIdx.x] = h[0][q] + h[1][q] + h[2][q] + h[3][q];
}

// Exclusive scan of each digit's per-block counts (digit-major rows of
// kSortBlocks counts, one block per digit, in place); tot[d] = the digit's
// total.  The scatter adds the digit bases (a scan of the totals) itself.
static_assert(kSortBlocks % NT == 0, "digit rows split evenly over the threads");
__global__ __launch_bounds__(NT) void k_radix_digit_scan(uint32_t* __restrict__ hist, uint32_t* __restrict__ tot) {
    constexpr int PER = kSortBlocks / NT;
    __shared__ uint32_t wsum[NT / 64];
    uint32_t* row = hist + (int64_t)blockIdx.x * kSortBlocks + threadIdx.x * PER;
    uint32_t v[PER], s = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        v[i] = row[i];
        s += v[i];
    }
    uint32_t all;
    uint32_t e = block_excl_scan(s, wsum, all);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        row[i] = e;
        e += v[i];
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = all;
}

// kGather (last pass only): 1 = instead of the keys, write gout[pos] =
// gsrc[value] (a per-value quantity wanted in sorted order); 2 = the same
// for the two elements 2 value, 2 value + 1 each value stands for, at
// positions 2 pos, 2 pos + 1 of vout and gout.
template <typename K, int BITS, int kGather>
__global__ __launch_bounds__(NT) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                      K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                      const int32_t* n_dev, int64_t n_host, int shift,
                                                      const uint32_t* __restrict__ offs,
                                                      const uint32_t* __restrict__ dtot,
                                                      const uint32_t* __restrict__ gsrc, uint32_t* __restrict__ gout) {
    constexpr int bits = BITS;
    constexpr int SORT_IPT = sort_ipt<K>(), SORT_TILE = sort_tile<K>(), SORT_WSEG = SORT_TILE / 4;
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t texcl[256];
    __shared__ uint32_t wsum[NT / 64];
    __shared__ K skey[SORT_TILE];
    __shared__ uint32_t sval[SORT_TILE];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t nbins = 1u << bits, mask = nbins - 1u;
    int64_t b0, b1;
    const int64_t n = count_of(n_dev, n_host);
    chunk_of(n, SORT_TILE, b0, b1);
    if (b0 >= b1) return;
    {
        // digit base (earlier digits' totals) + this block's prefix within the digit
        uint32_t all;
        const uint32_t dbase = block_excl_scan(threadIdx.x < nbins ? dtot[threadIdx.x] : 0u, wsum, all);
        if (threadIdx.x < nbins) run[threadIdx.x] = dbase + offs[(int64_t)threadIdx.x * gridDim.x + blockIdx.x];
    }
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int64_t base = b0; base < b1; base += SORT_TILE) {
        for (int i = threadIdx.x; i < 4 * 256; i += NT) (&cnt[0][0])[i] = 0u;
        __syncthreads();
        K key[SORT_IPT];
        uint32_t val[SORT_IPT], dg[SORT_IPT], lr[SORT_IPT];
        // issue every load of the sub-tile before any ranking work; a full
        // sub-tile needs no per-element bound
        const int64_t i0 = base + w * SORT_WSEG + lane;
        if (base + SORT_TILE <= b1) {
#pragma unroll
            for (int r = 0; r < SORT_IPT; ++r) {
                key[r] = kin[i0 + r * 64];
                val[r] = vin[i0 + r * 64];
            }
#pragma unroll
            for (int r = 0; r < SORT_IPT; ++r) dg[r] = digit(key[r], shift, mask);
        } else {
#pragma unroll
            for (int r = 0; r < SORT_IPT; ++r) {
                const bool valid = i0 + r * 64 < b1;
                key[r] = valid ? kin[i0 + r * 64] : (K)0;
                val[r] = valid ? vin[i0 + r * 64] : 0u;
                dg[r] = valid ? digit(key[r], shift, mask) : 0xffffffffu;
            }
        }
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            bool valid = dg[r] != 0xffffffffu;
            uint32_t d = valid ? dg[r] : 0u;
            uint64_t peers = peers_of<BITS>(d, valid);
            // every peer reads the wave's running count before the group's
            // first lane advances it (one wave, in-order LDS accesses)
            uint32_t c = valid ? cnt[w][d] : 0u;
            uint32_t rank = (uint32_t)__popcll(peers & lt);
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0u) cnt[w][d] = c + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            lr[r] = c + rank;
        }
        __syncthreads();
        uint32_t tot_d = 0;
        if (threadIdx.x < nbins) {
            uint32_t s = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t c = cnt[q][threadIdx.x];
                cnt[q][threadIdx.x] = s;
                s += c;
            }
            tot_d = s;
        }
        uint32_t all;
        uint32_t ex = block_excl_scan(tot_d, wsum, all);
        texcl[threadIdx.x] = ex;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SORT_IPT; ++r) {
            if (dg[r] != 0xffffffffu) {
                uint32_t lp = texcl[dg[r]] + cnt[w][dg[r]] + lr[r];
                skey[lp] = key[r];
                sval[lp] = val[r];
            }
        }
        __syncthreads();
        int n_tile = (int)(b1 - base < SORT_TILE ? b1 - base : SORT_TILE);
        for (int i = threadIdx.x; i < n_tile; i += NT) {
            K k = skey[i];
            uint32_t d = digit(k, shift, mask);
            const uint32_t pos = run[d] + (uint32_t)i - texcl[d];
            if ((int64_t)pos >= n) continue;  // never, for consistent counts; keeps writes in bounds
            const uint32_t v = sval[i];
            if (kGather == 2) {
                reinterpret_cast<uint2*>(gout)[pos] = reinterpret_cast<const uint2*>(gsrc)[v];
                reinterpret_cast<uint2*>(vout)[pos] = make_uint2(2u * v, 2u * v + 1u);
                continue;
            }
            if (kGather) gout[pos] = gsrc[v];
            else kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        if (threadIdx.x < nbins) run[threadIdx.x] += tot_d;
        __syncthreads();
    }
}

template <typename K>
void launch_scatter(int bits, const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, const int32_t* n_dev,
                    int64_t n_host, int shift, const uint32_t* offs, const uint32_t* dtot, const uint32_t* gsrc,
                    uint32_t* gout, bool pairs, hipStream_t st) {
    if (gout && pairs && bits == 8) {  // the depth sort's last pass
        hipLaunchKernelGGL((k_radix_scatter<K, 8, 2>), dim3(kSortBlocks), dim3(NT), 0, st, kin, vin, kout, vout, n_dev,
                           n_host, shift, offs, dtot, gsrc, gout);
        return;
    }
#define GSC_SCATTER(B)                                                                                               \
    if (gout)                                                                                                        \
        hipLaunchKernelGGL((k_radix_scatter<K, B, 1>), dim3(kSortBlocks), dim3(NT), 0, st, kin, vin, kout, vout,    \
                           n_dev, n_host, shift, offs, dtot, gsrc, gout);                                            \
    else                                                                                                             \
        hipLaunchKernelGGL((k_radix_scatter<K, B, 0>), dim3(kSortBlocks), dim3(NT), 0, st, kin, vin, kout, vout,    \
                           n_dev, n_host, shift, offs, dtot, gsrc, gout)
    switch (bits) {
        case 1: GSC_SCATTER(1); break;
        case 2: GSC_SCATTER(2); break;
        case 3: GSC_SCATTER(3); break;
        case 4: GSC_SCATTER(4); break;
        case 5: GSC_SCATTER(5); break;
        case 6: GSC_SCATTER(6); break;
        case 7: GSC_SCATTER(7); break;
        default: GSC_SCATTER(8); break;
    }
#undef GSC_SCATTER
}

template <typename K>
hipError_t radix_sort_impl(K* keys[2], uint32_t* vals[2], const int32_t* n_dev, int64_t n_host, int bit0, int bit1,
                           uint32_t* hist, uint32_t* block_sums, int* which, hipStream_t st, const uint32_t* gsrc,
                           uint32_t* gout, bool pairs) {
    if (pairs && (!gout || (bit1 - bit0) % 8 != 0)) return hipErrorInvalidValue;
    int cur = 0;
    for (int shift = bit0; shift < bit1; shift += 8) {
        int bits = bit1 - shift < 8 ? bit1 - shift : 8;
        hipLaunchKernelGGL(k_radix_hist<K>, dim3(kSortBlocks), dim3(NT), 0, st, keys[cur], n_dev, n_host, shift,
                           bits, hist);
        hipLaunchKernelGGL(k_radix_digit_scan, dim3(1u << bits), dim3(NT), 0, st, hist, block_sums);
        const bool last = shift + 8 >= bit1;
        launch_scatter<K>(bits, keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_dev, n_host, shift, hist,
                          block_sums, last ? gsrc : nullptr, last ? gout : nullptr, last && pairs, st);
        cur ^= 1;
    }
    *which = cur;
    return hipGetLastError();
}

}  // namespace

hipError_t scan_u32(const uint32_t* in, uint32_t* out, const int32_t* n_dev, int64_t n_host, int32_t* total,
                    uint32_t* block_sums, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(NT), 0, st, in, n_dev, n_host, block_sums);
    hipLaunchKernelGGL(k_scan_down, dim3(kScanBlocks), dim3(NT), 0, st, in, out, n_dev, n_host, block_sums, total);
    return hipGetLastError();
}

hipError_t scan_u64(const uint64_t* in, uint64_t* out, const int32_t* n_dev, int32_t* total_lo, int32_t* total_hi,
                    uint64_t* block_sums, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_reduce64, dim3(kScanBlocks), dim3(NT), 0, st, in, n_dev, block_sums);
    hipLaunchKernelGGL(k_scan_down64, dim3(kScanBlocks), dim3(NT), 0, st, in, out, n_dev, block_sums, total_lo,
                       total_hi);
    return hipGetLastError();
}

hipError_t compact_u32(const uint32_t* flags, const int32_t* n_dev, int64_t n_host, int32_t* total, int32_t* ids,
                       uint32_t* block_sums, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(NT), 0, st, flags, n_dev, n_host, block_sums);
    hipLaunchKernelGGL(k_scan_compact, dim3(kScanBlocks), dim3(NT), 0, st, flags, ids, n_dev, n_host, block_sums, total);
    return hipGetLastError();
}

hipError_t radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], const int32_t* n_dev, int64_t n_host, int bit0,
                          int bit1, uint32_t* hist, uint32_t* block_sums, int* which, hipStream_t st,
                          const uint32_t* gsrc, uint32_t* gout, bool pairs) {
    return radix_sort_impl<uint32_t>(keys, vals, n_dev, n_host, bit0, bit1, hist, block_sums, which, st, gsrc, gout,
                                     pairs);
}

hipError_t radix_sort_u16(uint16_t* keys[2], uint32_t* vals[2], const int32_t* n_dev, int64_t n_host, int bit0,
                          int bit1, uint32_t* hist, uint32_t* block_sums, int* which, hipStream_t st) {
    return radix_sort_impl<uint16_t>(keys, vals, n_dev, n_host, bit0, bit1, hist, block_sums, which, st, nullptr,
                                     nullptr, false);
}

hipError_t radix_sort_u64(uint64_t* keys[2], uint32_t* vals[2], const int32_t* n_dev, int64_t n_host, int bit0,
                          int bit1, uint32_t* hist, uint32_t* block_sums, int* which, hipStream_t st) {
    return radix_sort_impl<uint64_t>(keys, vals, n_dev, n_host, bit0, bit1, hist, block_sums, which, st, nullptr,
                                     nullptr, false);
}

}  // namespace gsc
