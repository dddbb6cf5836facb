// Derivation of missed anchors on MFMA (BF16 or FP8-weight forms).
#pragma once
#include <vector>

#include "gsc_common.h"

namespace gsc {

// Weight fragments in MFMA lane order, built on the host at load time.
// F32 (v_mfma_f32_16x16x4f32): layer 1 [6 hidden blocks][9 k-steps][64 lanes]
// floats; layer 2 [out tiles][2 hidden blocks][4 steps][64] floats.
// BF16 / FP8 (v_mfma_f32_16x16x16bf16_1k): layer 1 [6][3 k-blocks][64] x 4
// bf16; layer 2 [out tiles][2][64] x 4 bf16 (FP8 stores the e4m3 codes'
// exact bf16 values; the per-row scale multiplies the FP32 accumulator).
struct MfmaFrags {
    const float* l1_f32;
    const float* l2_f32;
    const uint16_t* l1_bf16;
    const uint16_t* l2_bf16;
    const uint16_t* l1_fp8;
    const uint16_t* l2_fp8;
    const float* b1;   // [96] layer-1 bias (hidden = head * 32 + r)
    const float* b2;   // [16 * n_tiles] layer-2 bias over padded outputs
    const float* s1;   // [96] FP8 row scales (layer 1)
    const float* s2;   // [16 * n_tiles] FP8 row scales (layer 2)
    int n_at, n_ct, n_vt;  // output tiles of the alpha, colour, covariance heads
};

// Host: pack fragments for k Gaussians per anchor from row-major weights
// W1[h] [32][n_in] (n_in = 35, or 36 with the distance input, which takes
// the padding column 35), W2[h] [c_h k][32], biases; returns host vectors to
// upload.
struct HostFrags {
    std::vector<float> l1_f32, l2_f32, b1, b2, s1, s2;
    std::vector<uint16_t> l1_bf16, l2_bf16, l1_fp8, l2_fp8;
    int n_at, n_ct, n_vt;
};
HostFrags pack_frags(const gsc_mlp& mlp, int k, int n_in);

struct MfmaDeriveArgs {
    const float4* posr;
    const float* feat;
    const float* scale;
    const float* offsets;
    int k;
    const int32_t* visible;
    const int32_t* misses;
    const int32_t* vslot;
    float4* L0;
    float4* L1;
    float4* L2;
    float* L3;
    uint16_t* line_mask;  // [lines] bit j: Gaussian j has alpha > 0 (may be null)
    float cam_pos[3];
    float inv_dist_unit;  // > 0: layer 1 takes |x - p_u| * inv_dist_unit as input 35
    const int32_t* n_miss;
    int mode;  // GSC_PREC_*
    MfmaFrags fr;
};

// Enqueue the MFMA derivation for up to n_max misses (count on the device).
hipError_t derive_mfma(const MfmaDeriveArgs& a, int64_t n_max, hipStream_t st);

}  // namespace gsc
