// BF16 inference of the reuse predictor (Linear 6-64-64-1, ReLU, sigmoid),
// shared by the cache lookup and the stand-alone inference entry point.
#pragma once
#include <cstdint>

#include "gsc_common.h"

namespace gsc {

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Two floats rounded to BF16 (nearest-even) and packed low | high << 16.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    uint32_t a = __float_as_uint(lo), b = __float_as_uint(hi);
    a += 0x7fffu + ((a >> 16) & 1u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (a >> 16) | (b & 0xffff0000u);
}

// acc + w.lo * h.lo + w.hi * h.hi (BF16 pairs, FP32 accumulation).
__device__ __forceinline__ float dot2_bf16(uint32_t w, uint32_t h, float acc) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w), __builtin_bit_cast(bf16x2_t, h), acc,
                                           false);
}

// p(stale) with BF16 weights and activations, FP32 accumulation: packed
// two-element dot products (weights as adjacent BF16 pairs of a row).
__device__ __forceinline__ float pred_prob_bf16(const uint16_t* __restrict__ wb, const float* __restrict__ w32, const float* f) {
    // layout: W1[64*6] b1[64] W2[64*64] b2[64] W3[64] b3[1]; every row starts at an even index
    const int oW1 = 0, ob1 = 64 * 6, oW2 = ob1 + 64, ob2 = oW2 + 64 * 64, oW3 = ob2 + 64, ob3 = oW3 + 64;
    // weights are read-only and the same for every lane: constant address
    // space, so they come through scalar loads
    typedef const __attribute__((address_space(4))) uint32_t* cwp_t;
    const cwp_t wp = (cwp_t)(const void*)wb;
    uint32_t x2[kPredIn / 2];
#pragma unroll
    for (int i = 0; i < kPredIn / 2; ++i) x2[i] = pack_bf16x2(f[2 * i], f[2 * i + 1]);
    uint32_t h1[kPredW / 2];
#pragma unroll
    for (int r = 0; r < kPredW; r += 2) {
        float a0 = w32[ob1 + r], a1 = w32[ob1 + r + 1];
#pragma unroll
        for (int c = 0; c < kPredIn / 2; ++c) {
            a0 = dot2_bf16(wp[(oW1 + r * kPredIn) / 2 + c], x2[c], a0);
            a1 = dot2_bf16(wp[(oW1 + (r + 1) * kPredIn) / 2 + c], x2[c], a1);
        }
        h1[r / 2] = pack_bf16x2(fmaxf(a0, 0.f), fmaxf(a1, 0.f));
    }
    float logit = w32[ob3];
    for (int r = 0; r < kPredW; r += 2) {
        float a0 = w32[ob2 + r], a1 = w32[ob2 + r + 1];
#pragma unroll
        for (int c = 0; c < kPredW / 2; ++c) {
            a0 = dot2_bf16(wp[(oW2 + r * kPredW) / 2 + c], h1[c], a0);
            a1 = dot2_bf16(wp[(oW2 + (r + 1) * kPredW) / 2 + c], h1[c], a1);
        }
        logit = dot2_bf16(wp[(oW3 + r) / 2], pack_bf16x2(fmaxf(a0, 0.f), fmaxf(a1, 0.f)), logit);
    }
    return 1.0f / (1.0f + expf(-logit));
}

}  // namespace gsc
