// BF16 inference of the reuse predictor (Linear 6-64-64-1, ReLU, sigmoid),
// one candidate per lane of a wave, shared by the cache lookup and the
// stand-alone inference entry point.
#pragma once
#include <cstdint>

#include "gsc_common.h"

namespace gsc {

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Two floats rounded to BF16 (nearest-even) and packed low | high << 16
// (one hardware conversion of the pair).
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// acc + w.lo * h.lo + w.hi * h.hi (BF16 pairs, FP32 accumulation).
__device__ __forceinline__ float dot2_bf16(uint32_t w, uint32_t h, float acc) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w), __builtin_bit_cast(bf16x2_t, h), acc,
                                           false);
}

typedef float pred_floatx4 __attribute__((ext_vector_type(4)));
typedef short pred_shortx4 __attribute__((ext_vector_type(4)));

// LDS the wave-level predictor needs per wave (dwords): one row of 32 packed
// BF16 hidden units per lane, padded to 34 dwords so that the 16 rows an
// 8-byte fragment read touches fall on distinct banks.
constexpr int kPredLdsStride = 34;
constexpr int kPredLdsWave = 64 * kPredLdsStride;

// BF16 value rounded from x (nearest-even), as a float.
__device__ __forceinline__ float round_bf16(float x) { return (float)(__bf16)x; }

// p(stale) of the wave's 64 candidates (the features f of this lane's),
// BF16 weights and activations, FP32 accumulation.
//   layer 1 per lane: packed two-element BF16 dot products, the hidden
//     vector rounded to BF16 and stored in this lane's row of `lds`;
//   layer 2 on the matrix cores, O = W2 H over the wave: M = 64 output
//     units, K = 64 hidden units, N = the 64 candidates, in 16x16x16 BF16
//     tiles (A: W2 rows from memory; B: hidden vectors read back from `lds`,
//     i.e. transposed); bias, ReLU and BF16 rounding on the FP32 result;
//   layer 3 as per-lane partial sums over the output rows a lane holds, added
//     across the four row groups of a column (lanes c, c^16, c^32, c^48).
// Every lane of the wave must call it (the matrix instructions run on the
// whole wave); a lane without a candidate passes any finite features and
// ignores the result.  `lds`: kPredLdsWave dwords of this wave.
__device__ __forceinline__ float pred_prob_bf16_wave(const uint16_t* __restrict__ wb, const float* __restrict__ w32,
                                                     const float* f, uint32_t* lds) {
    // layout: W1[64*6] b1[64] W2[64*64] b2[64] W3[64] b3[1]; every row starts at an even index
    const int oW1 = 0, ob1 = 64 * 6, oW2 = ob1 + 64, ob2 = oW2 + 64 * 64, oW3 = ob2 + 64, ob3 = oW3 + 64;
    // uniform weights and biases through the constant address space (scalar loads)
    typedef const __attribute__((address_space(4))) uint32_t* cwp_t;
    typedef const __attribute__((address_space(4))) float* cfp_t;
    const cwp_t wp = (cwp_t)(const void*)wb;
    const cfp_t wf = (cfp_t)(const void*)w32;
    const int lane = threadIdx.x & 63, col = lane & 15, q = lane >> 4;
    uint32_t x2[kPredIn / 2];
#pragma unroll
    for (int i = 0; i < kPredIn / 2; ++i) x2[i] = pack_bf16x2(f[2 * i], f[2 * i + 1]);
    uint32_t* row = lds + lane * kPredLdsStride;
#pragma unroll
    for (int r = 0; r < kPredW; r += 2) {
        float a0 = wf[ob1 + r], a1 = wf[ob1 + r + 1];
#pragma unroll
        for (int c = 0; c < kPredIn / 2; ++c) {
            a0 = dot2_bf16(wp[(oW1 + r * kPredIn) / 2 + c], x2[c], a0);
            a1 = dot2_bf16(wp[(oW1 + (r + 1) * kPredIn) / 2 + c], x2[c], a1);
        }
        row[r / 2] = pack_bf16x2(fmaxf(a0, 0.f), fmaxf(a1, 0.f));
    }
    __builtin_amdgcn_wave_barrier();  // a wave's LDS accesses complete in issue order
    // B fragments: candidate 16 nt + col, hidden units 16 ks + 4 q .. + 3
    pred_shortx4 B[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            B[nt][ks] = __builtin_bit_cast(pred_shortx4,
                                           *reinterpret_cast<const uint2*>(lds + (nt * 16 + col) * kPredLdsStride +
                                                                           ks * 8 + 2 * q));
    __builtin_amdgcn_wave_barrier();  // read before the caller writes the rows again
    const uint2* W2 = reinterpret_cast<const uint2*>(wb + oW2);     // 4 BF16 per element
    const uint2* W3 = reinterpret_cast<const uint2*>(wb + oW3);
    const float4* b2 = reinterpret_cast<const float4*>(w32 + ob2);
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        pred_floatx4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = pred_floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            // A fragment: output unit 16 mt + col, hidden units 16 ks + 4 q .. + 3
            const pred_shortx4 A = __builtin_bit_cast(pred_shortx4, W2[((mt * 16 + col) * 64 + ks * 16 + 4 * q) / 4]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B[nt][ks], acc[nt], 0, 0, 0);
        }
        // acc[nt][i]: output unit 16 mt + 4 q + i of candidate 16 nt + col
        const float4 bb = b2[mt * 4 + q];
        const uint2 w3 = W3[mt * 4 + q];
        const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
        const float wv[4] = {__uint_as_float(w3.x << 16), __uint_as_float(w3.x & 0xffff0000u),
                             __uint_as_float(w3.y << 16), __uint_as_float(w3.y & 0xffff0000u)};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) part[nt] = fmaf(wv[i], round_bf16(fmaxf(acc[nt][i] + bv[i], 0.f)), part[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        part[nt] += __shfl_xor(part[nt], 16, 64);
        part[nt] += __shfl_xor(part[nt], 32, 64);
    }
    // candidate `lane` is column lane & 15 of tile lane >> 4
    const float mine = q == 0 ? part[0] : (q == 1 ? part[1] : (q == 2 ? part[2] : part[3]));
    const float logit = wf[ob3] + mine;
    return 1.0f / (1.0f + expf(-logit));
}

}  // namespace gsc
