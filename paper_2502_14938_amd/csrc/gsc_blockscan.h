// Block-level pieces of the device-wide scans (256-thread blocks, wave64):
// the generic scan and compaction kernels use them, and so do scans fused
// with the work that produces their input or consumes their output (the
// composition of the render buffer).  A scan runs as a reduce pass (one sum
// per block) and a down-sweep; every block owns one contiguous chunk of the
// input, whose length it reads from device memory.
#pragma once
#include <cstdint>

#include "gsc_common.h"

namespace gsc {
namespace blockscan {

constexpr int kThreads = 256;
constexpr int kTile = 1024;  // elements per down-sweep step (4 per thread)

__device__ __forceinline__ int64_t count_of(const int32_t* n_dev, int64_t n_host) {
    return n_dev ? (int64_t)(*n_dev) : n_host;
}

// This block's chunk [b0, b1) of n elements, chunks aligned to `align`.
__device__ __forceinline__ void chunk_of(int64_t n, int64_t align, int64_t& b0, int64_t& b1) {
    int64_t per = (n + gridDim.x - 1) / gridDim.x;
    per = (per + align - 1) / align * align;
    b0 = (int64_t)blockIdx.x * per;
    b1 = b0 + per < n ? b0 + per : n;
}

// Exclusive scan across the 256 threads of a block (one value each); T is
// uint32_t or uint64_t (two 32-bit counts packed in one value add
// independently while neither field overflows).
template <typename T = uint32_t>
__device__ __forceinline__ T block_excl_scan(T v, T* wsum, T& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) {
        T s = wsum[i];
        pre += i < w ? s : (T)0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

template <typename T = uint32_t>
__device__ __forceinline__ T block_sum(T v, T* wsum) {
    T t;
    block_excl_scan<T>(v, wsum, t);
    return t;
}

// Down-sweep carry of this block: the sum of the preceding blocks' sums (at
// most gridDim.x values, a block reduction, so no pass over the block sums
// of its own); the last block also writes the total (when asked).
template <typename T = uint32_t>
__device__ __forceinline__ T block_carry(const T* __restrict__ block_sums, T* wsum) {
    T part = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kThreads) part += block_sums[i];
    return block_sum<T>(part, wsum);
}

__device__ __forceinline__ uint32_t block_carry(const uint32_t* __restrict__ block_sums, uint32_t* wsum,
                                                int32_t* total) {
    const uint32_t carry = block_carry<uint32_t>(block_sums, wsum);
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = (int32_t)(carry + block_sums[blockIdx.x]);
    return carry;
}

}  // namespace blockscan
}  // namespace gsc
