// Derivation of missed anchors on MFMA (BF16 or FP8-weight forms).
#pragma once
#include "gsc_common.h"

namespace gsc {

struct MfmaDeriveArgs {
    const float4* posr;
    const float* feat;
    const float* scale;
    const float* offsets;
    const float* w32;         // fp32 weights (biases are read from here)
    const uint16_t* wbf16;    // bf16 weights, same layout
    const uint8_t* wfp8;      // e4m3fn weights, same layout
    const float* wfp8_scale;  // per output row
    WeightLayout L;
    int k;
    const int32_t* visible;
    const int32_t* misses;
    const int32_t* vslot;
    float4* L0;
    float4* L1;
    float4* L2;
    float* L3;
    float cam_pos[3];
    const int32_t* n_miss;
    int fp8;
};

// Enqueue the MFMA derivation for up to n_max misses (count on the device).
hipError_t derive_mfma(const MfmaDeriveArgs& a, int64_t n_max, hipStream_t st);

}  // namespace gsc
