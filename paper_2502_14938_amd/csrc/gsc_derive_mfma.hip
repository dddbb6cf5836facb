// Derivation of missed anchors on the matrix cores (Section 3.1 eq. 3; the
// AnchorDecoder of Section 6: the anchor row is read once for all k offsets,
// both MLP layers run back to back without leaving registers, and every
// output attribute is written straight into its cache array).
//
// One wave handles 16 anchors.  Layer 1 is computed transposed,
// H^T[96 x 16] = W1[96 x 35] Z^T[35 x 16], so that each 16x16 output tile is
// already laid out as the B operand of layer 2, O^T = W2 H^T.  The 110
// outputs of the anchor (alpha k, colour 3k, covariance 7k) land in LDS and
// an epilogue turns them into the k Gaussians (activations, quaternion,
// Sigma = R S S^T R^T (eq. 2), mean = x + s * O_j).
//
// MODE GSC_PREC_F32: v_mfma_f32_16x16x4f32 (FP32 operands, FP32 accumulate).
// MODE GSC_PREC_BF16: v_mfma_f32_16x16x16bf16_1k, inputs and hidden
//   activations rounded to bfloat16 (nearest even), FP32 accumulate.
// MODE GSC_PREC_FP8: as BF16 with e4m3fn weights (exact in bfloat16) and a
//   per-output-row FP32 scale applied to the accumulator.
#include <cmath>
#include <cstring>

#include "gsc_derive_mfma.h"

namespace gsc {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;
constexpr int kMaxOutTiles = 11;            // ceil(k/16) + ceil(3k/16) + ceil(7k/16) for k <= 16
constexpr int kOutPad = 16 * kMaxOutTiles;  // padded outputs per anchor

uint16_t h_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float h_from_bf16(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// e4m3fn value nearest to x (ties to even), saturating at 448.
double h_e4m3(double x) {
    if (x == 0.0) return 0.0;
    double a = std::fabs(x), r;
    if (a < std::ldexp(1.0, -6)) {
        r = std::nearbyint(a / std::ldexp(1.0, -9)) * std::ldexp(1.0, -9);
    } else {
        int e;
        std::frexp(a, &e);
        double q = std::ldexp(1.0, e - 4);
        r = std::nearbyint(a / q) * q;
    }
    if (r > 448.0) r = 448.0;
    return x < 0 ? -r : r;
}

__device__ __forceinline__ short d_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

}  // namespace

HostFrags pack_frags(const gsc_mlp& mlp, int k, int n_in) {
    HostFrags f;
    const int c[3] = {1, 3, 7};
    f.n_at = (k + 15) / 16;
    f.n_ct = (3 * k + 15) / 16;
    f.n_vt = (7 * k + 15) / 16;
    const int nt = f.n_at + f.n_ct + f.n_vt;
    const int tile0[3] = {0, f.n_at, f.n_at + f.n_ct};
    // layer 1, padded [96][48]; scales per hidden row
    std::vector<double> W1p(96 * 48, 0.0), q1(96 * 48, 0.0);
    f.b1.assign(96, 0.f);
    f.s1.assign(96, 1.f);
    for (int h = 0; h < 3; ++h)
        for (int r = 0; r < 32; ++r) {
            int row = h * 32 + r;
            double amax = 0.0;
            for (int q = 0; q < n_in; ++q) {
                W1p[row * 48 + q] = mlp.W1[h][r * n_in + q];
                amax = std::fmax(amax, std::fabs(W1p[row * 48 + q]));
            }
            double s = amax > 0.0 ? amax / 448.0 : 1.0;
            f.s1[row] = (float)s;
            for (int q = 0; q < n_in; ++q) q1[row * 48 + q] = h_e4m3(W1p[row * 48 + q] / s);
            f.b1[row] = mlp.b1[h][r];
        }
    // layer 2, padded [16 nt][32] per tile's head
    std::vector<double> W2p(16 * nt * 32, 0.0), q2(16 * nt * 32, 0.0);
    f.b2.assign(16 * nt, 0.f);
    f.s2.assign(16 * nt, 1.f);
    for (int h = 0; h < 3; ++h)
        for (int o = 0; o < c[h] * k; ++o) {
            int row = 16 * tile0[h] + o;
            double amax = 0.0;
            for (int q = 0; q < 32; ++q) {
                W2p[row * 32 + q] = mlp.W2[h][o * 32 + q];
                amax = std::fmax(amax, std::fabs(W2p[row * 32 + q]));
            }
            double s = amax > 0.0 ? amax / 448.0 : 1.0;
            f.s2[row] = (float)s;
            for (int q = 0; q < 32; ++q) q2[row * 32 + q] = h_e4m3(W2p[row * 32 + q] / s);
            f.b2[row] = mlp.b2[h][o];
        }
    // F32 fragments
    f.l1_f32.assign(6 * 9 * 64, 0.f);
    for (int hb = 0; hb < 6; ++hb)
        for (int ks = 0; ks < 9; ++ks)
            for (int l = 0; l < 64; ++l) {
                int row = hb * 16 + (l & 15), col = 4 * ks + (l >> 4);
                f.l1_f32[(hb * 9 + ks) * 64 + l] = col < n_in ? (float)W1p[row * 48 + col] : 0.f;
            }
    f.l2_f32.assign(nt * 2 * 4 * 64, 0.f);
    for (int ot = 0; ot < nt; ++ot)
        for (int hb2 = 0; hb2 < 2; ++hb2)
            for (int s = 0; s < 4; ++s)
                for (int l = 0; l < 64; ++l) {
                    int row = ot * 16 + (l & 15), col = 16 * hb2 + 4 * (l >> 4) + s;
                    f.l2_f32[((ot * 2 + hb2) * 4 + s) * 64 + l] = (float)W2p[row * 32 + col];
                }
    // BF16 / FP8 fragments: 4 consecutive k per lane
    f.l1_bf16.assign(6 * 3 * 64 * 4, 0);
    f.l1_fp8.assign(6 * 3 * 64 * 4, 0);
    for (int hb = 0; hb < 6; ++hb)
        for (int kb = 0; kb < 3; ++kb)
            for (int l = 0; l < 64; ++l)
                for (int i = 0; i < 4; ++i) {
                    int row = hb * 16 + (l & 15), col = 16 * kb + 4 * (l >> 4) + i;
                    size_t at = ((size_t)(hb * 3 + kb) * 64 + l) * 4 + i;
                    f.l1_bf16[at] = h_bf16((float)W1p[row * 48 + col]);
                    f.l1_fp8[at] = h_bf16((float)q1[row * 48 + col]);
                }
    f.l2_bf16.assign(nt * 2 * 64 * 4, 0);
    f.l2_fp8.assign(nt * 2 * 64 * 4, 0);
    for (int ot = 0; ot < nt; ++ot)
        for (int kb = 0; kb < 2; ++kb)
            for (int l = 0; l < 64; ++l)
                for (int i = 0; i < 4; ++i) {
                    int row = ot * 16 + (l & 15), col = 16 * kb + 4 * (l >> 4) + i;
                    size_t at = ((size_t)(ot * 2 + kb) * 64 + l) * 4 + i;
                    f.l2_bf16[at] = h_bf16((float)W2p[row * 32 + col]);
                    f.l2_fp8[at] = h_bf16((float)q2[row * 32 + col]);
                }
    (void)h_from_bf16;
    return f;
}

namespace {

template <int MODE>
__global__ __launch_bounds__(NT) void k_derive_mfma(MfmaDeriveArgs a) {
    __shared__ float O[4][16][kOutPad + 1];
    __shared__ int32_t sAid[4][16];
    __shared__ int32_t sLine[4][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const MfmaFrags& fr = a.fr;
    const int nt = fr.n_at + fr.n_ct + fr.n_vt;
    const int k = a.k;
    // layer-1 weights stay in registers for the whole kernel
    float w1f[(MODE == GSC_PREC_F32) ? 54 : 1];
    shortx4 w1h[(MODE == GSC_PREC_F32) ? 1 : 18];
    if (MODE == GSC_PREC_F32) {
#pragma unroll
        for (int i = 0; i < 54; ++i) w1f[i] = fr.l1_f32[i * 64 + lane];
    } else {
        const uint16_t* src = MODE == GSC_PREC_BF16 ? fr.l1_bf16 : fr.l1_fp8;
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            const uint2 v = reinterpret_cast<const uint2*>(src)[i * 64 + lane];
            w1h[i] = shortx4{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff), (short)(v.y >> 16)};
        }
    }
    const int32_t n = *a.n_miss;
    const int ntiles = (n + 15) / 16;
    for (int t0 = blockIdx.x * 4; t0 < ntiles; t0 += gridDim.x * 4) {
        const int tile = t0 + w;
        if (tile < ntiles) {
            const int m = tile * 16 + col;
            const bool ok = m < n;
            int32_t pos = ok ? a.misses[m] : 0;
            int32_t aid = ok ? a.visible[pos] : 0;
            int32_t line = ok ? a.vslot[pos] : -1;
            if (q == 0) {
                sAid[w][col] = aid;
                sLine[w][col] = line;
            }
            const float4 x = a.posr[aid];
            float vx = x.x - a.cam_pos[0], vy = x.y - a.cam_pos[1], vz = x.z - a.cam_pos[2];
            const float nv = sqrtf(vx * vx + vy * vy + vz * vz);
            const float inv = 1.0f / nv;
            const float dv[3] = {vx * inv, vy * inv, vz * inv};
            // the optional distance input (column 35; its weights are zero without it)
            const float dn = a.inv_dist_unit > 0.f ? nv * a.inv_dist_unit : 0.f;
            const float* f = a.feat + (int64_t)aid * kF;
            // ---- layer 1: H^T = W1 Z^T, 6 tiles of 16 hidden units
            floatx4 acc[6];
#pragma unroll
            for (int hb = 0; hb < 6; ++hb) acc[hb] = floatx4{0.f, 0.f, 0.f, 0.f};
            if (MODE == GSC_PREC_F32) {
#pragma unroll
                for (int ks = 0; ks < 9; ++ks) {
                    int in = 4 * ks + q;
                    float b = in < kF ? f[in] : (in < kF + 3 ? dv[in - kF] : (in == kF + 3 ? dn : 0.f));
#pragma unroll
                    for (int hb = 0; hb < 6; ++hb)
                        acc[hb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1f[hb * 9 + ks], b, acc[hb], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int kb = 0; kb < 3; ++kb) {
                    float z[4];
                    if (kb < 2) {
                        float4 v = reinterpret_cast<const float4*>(f)[kb * 4 + q];
                        z[0] = v.x; z[1] = v.y; z[2] = v.z; z[3] = v.w;
                    } else {
                        z[0] = q == 0 ? dv[0] : 0.f;
                        z[1] = q == 0 ? dv[1] : 0.f;
                        z[2] = q == 0 ? dv[2] : 0.f;
                        z[3] = q == 0 ? dn : 0.f;
                    }
                    shortx4 b = shortx4{d_bf16(z[0]), d_bf16(z[1]), d_bf16(z[2]), d_bf16(z[3])};
#pragma unroll
                    for (int hb = 0; hb < 6; ++hb)
                        acc[hb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1h[hb * 3 + kb], b, acc[hb], 0, 0, 0);
                }
            }
            // bias + ReLU (rows hb*16 + 4q + i of H^T, column = this lane's anchor)
            float h[6][4];
            shortx4 hh[6];
#pragma unroll
            for (int hb = 0; hb < 6; ++hb) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int row = hb * 16 + 4 * q + i;
                    float v = acc[hb][i];
                    if (MODE == GSC_PREC_FP8) v *= fr.s1[row];
                    h[hb][i] = fmaxf(v + fr.b1[row], 0.f);
                }
                if (MODE != GSC_PREC_F32)
                    hh[hb] = shortx4{d_bf16(h[hb][0]), d_bf16(h[hb][1]), d_bf16(h[hb][2]), d_bf16(h[hb][3])};
            }
            // ---- layer 2: O^T = W2 H^T per 16-output tile
            for (int ot = 0; ot < nt; ++ot) {
                const int head = ot < fr.n_at ? 0 : (ot < fr.n_at + fr.n_ct ? 1 : 2);
                floatx4 o = floatx4{0.f, 0.f, 0.f, 0.f};
                if (MODE == GSC_PREC_F32) {
#pragma unroll
                    for (int hb2 = 0; hb2 < 2; ++hb2)
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            float av = fr.l2_f32[((ot * 2 + hb2) * 4 + s) * 64 + lane];
                            float bv = head == 0 ? h[hb2][s] : (head == 1 ? h[2 + hb2][s] : h[4 + hb2][s]);
                            o = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, o, 0, 0, 0);
                        }
                } else {
                    const uint16_t* src = MODE == GSC_PREC_BF16 ? fr.l2_bf16 : fr.l2_fp8;
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb) {
                        const uint2 v = reinterpret_cast<const uint2*>(src)[(ot * 2 + kb) * 64 + lane];
                        shortx4 av = shortx4{(short)(v.x & 0xffff), (short)(v.x >> 16), (short)(v.y & 0xffff),
                                             (short)(v.y >> 16)};
                        shortx4 bv = head == 0 ? hh[kb] : (head == 1 ? hh[2 + kb] : hh[4 + kb]);
                        o = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, o, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int row = ot * 16 + 4 * q + i;
                    float v = o[i];
                    if (MODE == GSC_PREC_FP8) v *= fr.s2[row];
                    O[w][col][row] = v + fr.b2[row];
                }
            }
        }
        __syncthreads();
        if (tile < ntiles) {
            // ---- epilogue: one Gaussian per lane step
            const int cbase = 16 * fr.n_at, vbase = 16 * (fr.n_at + fr.n_ct);
            for (int g = lane; g < 16 * k; g += 64) {
                const int al = g / k, j = g - al * k;
                const int m = tile * 16 + al;
                const int32_t line = sLine[w][al];
                if (m >= n || line < 0) continue;
                const int32_t aid = sAid[w][al];
                const float* Ov = O[w][al];
                const float4 x = a.posr[aid];
                const float* sc = a.scale + (int64_t)aid * 6;
                const float* off = a.offsets + ((int64_t)aid * k + j) * 3;
                float alpha = tanhf(Ov[j]);
                float r = sigm(Ov[cbase + 3 * j]), gg = sigm(Ov[cbase + 3 * j + 1]), bb = sigm(Ov[cbase + 3 * j + 2]);
                const float* os = Ov + vbase + 7 * j;
                float s0 = sc[3] * sigm(os[0]), s1 = sc[4] * sigm(os[1]), s2 = sc[5] * sigm(os[2]);
                float qw = os[3], qx = os[4], qy = os[5], qz = os[6];
                float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
                if (qn > 0.f) {
                    float iq = 1.0f / qn;
                    qw *= iq; qx *= iq; qy *= iq; qz *= iq;
                } else {
                    qw = 1.f; qx = qy = qz = 0.f;
                }
                float R[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
                                 {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
                                 {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
                float v[3] = {s0 * s0, s1 * s1, s2 * s2};
                float S[6];
                int idx = 0;
#pragma unroll
                for (int rr = 0; rr < 3; ++rr)
#pragma unroll
                    for (int cc = rr; cc < 3; ++cc)
                        S[idx++] = R[rr][0] * v[0] * R[cc][0] + R[rr][1] * v[1] * R[cc][1] + R[rr][2] * v[2] * R[cc][2];
                const int64_t e = (int64_t)line * k + j;
                // position relative to the anchor (small, so FP32 keeps it to
                // ~1e-7 m); the rasteriser adds anchor - camera in FP64
                a.L0[e] = make_float4(sc[0] * off[0], sc[1] * off[1], sc[2] * off[2], alpha);
                a.L1[e] = make_float4(S[0], S[1], S[2], S[3]);
                a.L2[e] = make_float4(S[4], S[5], r, gg);
                a.L3[e] = bb;
            }
            // the line's mask of kept Gaussians (alpha > 0, the render
            // buffer's test), from the same alphas
            if (a.line_mask && lane < 16) {
                const int m = tile * 16 + lane;
                const int32_t line = sLine[w][lane];
                if (m < n && line >= 0) {
                    uint32_t mk = 0;
                    for (int j = 0; j < k; ++j) mk |= tanhf(O[w][lane][j]) > 0.f ? 1u << j : 0u;
                    a.line_mask[line] = (uint16_t)mk;
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t derive_mfma(const MfmaDeriveArgs& a, int64_t n_max, hipStream_t st) {
    int64_t tiles = (n_max + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > kGridBlocks) blocks = kGridBlocks;
    switch (a.mode) {
        case GSC_PREC_F32:
            hipLaunchKernelGGL(k_derive_mfma<GSC_PREC_F32>, dim3((unsigned)blocks), dim3(NT), 0, st, a);
            break;
        case GSC_PREC_BF16:
            hipLaunchKernelGGL(k_derive_mfma<GSC_PREC_BF16>, dim3((unsigned)blocks), dim3(NT), 0, st, a);
            break;
        default:
            hipLaunchKernelGGL(k_derive_mfma<GSC_PREC_FP8>, dim3((unsigned)blocks), dim3(NT), 0, st, a);
            break;
    }
    return hipGetLastError();
}

}  // namespace gsc
