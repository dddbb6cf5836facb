// Image-quality metric on the device: mean SSIM of two CHW float images
// (the third metric of the quality table, Table 4; Wang et al. 2004).
//
// Per channel, local means, variances and covariance under an 11 x 11
// Gaussian window (sigma 1.5, normalised), constants C1 = 0.01^2 and
// C2 = 0.03^2 (dynamic range 1), the SSIM map over every window position
// inside the image, averaged over positions and channels.
//
//   k_ssim        one block per 16 x 16 tile of window positions and channel:
//                 the 26 x 26 patch of both images in LDS, the five
//                 horizontal window sums per patch row, then the vertical
//                 sums and the map value per position, all in FP64 (the
//                 variances are differences of nearly equal sums, and FP64
//                 vector FMA runs at the non-packed FP32 rate); the block's
//                 sum to its own slot
//   k_ssim_total  one block adds the slots in a fixed order (deterministic)
#include <cmath>

#include "gsc_common.h"
#include "gsc_ctx.h"

namespace gsc {

namespace {

constexpr int kWin = 11;
constexpr int kTileS = 16;
constexpr int kPatch = kTileS + kWin - 1;
constexpr int kThreads = kTileS * kTileS;  // one window position per thread

__global__ __launch_bounds__(kThreads) void k_ssim(const float* __restrict__ a, const float* __restrict__ b, int H,
                                                   int W, SsimWindow win, int tiles_x, double* __restrict__ partial) {
    __shared__ float sa[kPatch][kPatch + 1];
    __shared__ float sb[kPatch][kPatch + 1];
    __shared__ double hs[5][kPatch][kTileS + 1];  // horizontal sums: mean a, mean b, a^2, b^2, ab
    __shared__ double wsum[kThreads / 64];
    const int ch = blockIdx.y;
    const int x0 = (blockIdx.x % tiles_x) * kTileS, y0 = (blockIdx.x / tiles_x) * kTileS;
    const int64_t plane = (int64_t)H * W;
    const float* A = a + ch * plane;
    const float* B = b + ch * plane;
    for (int i = threadIdx.x; i < kPatch * kPatch; i += kThreads) {
        const int r = i / kPatch, c = i % kPatch, y = y0 + r, x = x0 + c;
        const bool in = y < H && x < W;
        sa[r][c] = in ? A[(int64_t)y * W + x] : 0.f;
        sb[r][c] = in ? B[(int64_t)y * W + x] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kPatch * kTileS; i += kThreads) {
        const int r = i / kTileS, j = i % kTileS;
        double m1 = 0.0, m2 = 0.0, s11 = 0.0, s22 = 0.0, s12 = 0.0;
#pragma unroll
        for (int t = 0; t < kWin; ++t) {
            const double x = sa[r][j + t], y = sb[r][j + t], w = win.w[t];
            m1 = fma(w, x, m1);
            m2 = fma(w, y, m2);
            s11 = fma(w, x * x, s11);
            s22 = fma(w, y * y, s22);
            s12 = fma(w, x * y, s12);
        }
        hs[0][r][j] = m1; hs[1][r][j] = m2; hs[2][r][j] = s11; hs[3][r][j] = s22; hs[4][r][j] = s12;
    }
    __syncthreads();
    const int oy = threadIdx.x / kTileS, ox = threadIdx.x % kTileS;
    double v = 0.0;
    if (y0 + oy <= H - kWin && x0 + ox <= W - kWin) {
        double m1 = 0.0, m2 = 0.0, s11 = 0.0, s22 = 0.0, s12 = 0.0;
#pragma unroll
        for (int t = 0; t < kWin; ++t) {
            const double w = win.w[t];
            m1 = fma(w, hs[0][oy + t][ox], m1);
            m2 = fma(w, hs[1][oy + t][ox], m2);
            s11 = fma(w, hs[2][oy + t][ox], s11);
            s22 = fma(w, hs[3][oy + t][ox], s22);
            s12 = fma(w, hs[4][oy + t][ox], s12);
        }
        const double c1 = 1e-4, c2 = 9e-4;
        const double vx = s11 - m1 * m1, vy = s22 - m2 * m2, cxy = s12 - m1 * m2;
        v = ((2.0 * m1 * m2 + c1) * (2.0 * cxy + c2)) / ((m1 * m1 + m2 * m2 + c1) * (vx + vy + c2));
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kThreads / 64; ++q) t += wsum[q];
        partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(256) void k_ssim_total(const double* __restrict__ partial, int64_t n, double* out) {
    __shared__ double s[256];
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) t += partial[i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

}  // namespace

SsimWindow ssim_window() {
    SsimWindow win;
    double g[kWin], sum = 0.0;
    for (int i = 0; i < kWin; ++i) {
        const double x = i - 0.5 * (kWin - 1);
        g[i] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
        sum += g[i];
    }
    for (int i = 0; i < kWin; ++i) win.w[i] = g[i] / sum;
    return win;
}

int64_t ssim_blocks(int C, int H, int W) {
    const int64_t tx = (W - kWin + 1 + kTileS - 1) / kTileS, ty = (H - kWin + 1 + kTileS - 1) / kTileS;
    return tx * ty * C;
}

hipError_t ssim_launch(const float* a, const float* b, int C, int H, int W, const SsimWindow& win, double* partial,
                       double* total, hipStream_t st) {
    const int tiles_x = (W - kWin + 1 + kTileS - 1) / kTileS, tiles_y = (H - kWin + 1 + kTileS - 1) / kTileS;
    hipLaunchKernelGGL(k_ssim, dim3((unsigned)(tiles_x * tiles_y), (unsigned)C), dim3(kThreads), 0, st, a, b, H, W, win,
                       tiles_x, partial);
    hipLaunchKernelGGL(k_ssim_total, dim3(1), dim3(256), 0, st, partial, ssim_blocks(C, H, W), total);
    return hipGetLastError();
}

}  // namespace gsc
