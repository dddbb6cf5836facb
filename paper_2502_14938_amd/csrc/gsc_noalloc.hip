// Allocation-free raster-only entry (gsc_render_gaussians_noalloc): the
// rasterisation of explicit Gaussians (EWA projection, exact tile binning,
// sort, ranges, blend) with every intermediate buffer carved out of one
// file-scope device array instead of memory the library allocates, for
// callers that cannot allocate (HIP graph capture, tight serving loops).
//
// The array lives as long as the code object on each device that runs the
// library.  Host code never passes its name to a kernel: the name is a host
// stand-in, so its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// used.  Every call on a device shares that device's array, so calls that
// overlap on one device race; the kernels rewrite every counter they read
// (k_preprocess resets the batch counters and clears the tile ranges), so
// nothing has to start at zero.
#include <cstring>
#include <mutex>
#include <string>

#include "gsc_common.h"
#include "gsc_ctx.h"

namespace gsc {

namespace {

constexpr int64_t kNaTiles = (int64_t)(GSC_NOALLOC_MAX_SIDE / kTile) * (GSC_NOALLOC_MAX_SIDE / kTile);
constexpr size_t kNaBytes = (size_t)48 << 20;  // holds the layout below (checked at set-up)
constexpr size_t kNaAlign = 256;
constexpr int kNaDevices = 64;

__device__ __align__(256) uint8_t scratch[kNaBytes];

// Per device: the array's device address and the buffers carved from it.
struct NaDevice {
    bool ready = false;
    float4* L0 = nullptr;
    float4* L1 = nullptr;
    float4* L2 = nullptr;
    float* L3 = nullptr;
    Raster r;
};

std::mutex g_na_mu;
NaDevice g_na[kNaDevices];

// Bump allocation over the array (256-byte aligned pieces).
struct Carve {
    uint8_t* base;
    size_t used = 0;
    size_t cap;
    template <typename T>
    hipError_t operator()(T*& p, int64_t count) {
        const size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
        used = (used + kNaAlign - 1) / kNaAlign * kNaAlign;
        if (used + bytes > cap) return hipErrorOutOfMemory;
        p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return hipSuccess;
    }
};

// Once per device, with that device current: the array's address, then the
// layout (the raster buffers for GSC_NOALLOC_MAX_GAUSSIANS entries,
// GSC_NOALLOC_MAX_PAIRS pairs and the tiles of a GSC_NOALLOC_MAX_SIDE square
// image, after the Gaussians' four line arrays).
int na_setup(int dev, NaDevice*& out) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    NaDevice& d = g_na[dev];
    if (!d.ready) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return global_fail(GSC_E_HIP, std::string("gsc_render_gaussians_noalloc: hipGetSymbolAddress: ") +
                                              hipGetErrorString(e));
        Carve cv{static_cast<uint8_t*>(ptr), 0, kNaBytes};
        const int64_t n = GSC_NOALLOC_MAX_GAUSSIANS;
        NaDevice t;
        if (cv(t.L0, n) != hipSuccess || cv(t.L1, n) != hipSuccess || cv(t.L2, n) != hipSuccess ||
            cv(t.L3, n) != hipSuccess ||
            raster_layout(t.r, n, GSC_NOALLOC_MAX_PAIRS, kNaTiles, false, cv) != hipSuccess)
            return global_fail(GSC_E_HIP, "gsc_render_gaussians_noalloc: the static buffer is too small for its layout");
        t.r.max_entries = n;
        t.r.max_pairs = GSC_NOALLOC_MAX_PAIRS;
        t.r.max_tiles = kNaTiles;
        t.r.srow_cap = n;
        t.r.tall_cap = n / 4 + 256;
        t.r.cnt_host = nullptr;  // counters are read on the device only
        t.ready = true;
        d = t;
    }
    out = &d;
    return GSC_OK;
}

__global__ void k_na_status(const RasterCounters* rc, int32_t* status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = rc->overflow;
}

bool na_camera_ok(const gsc_camera& c) {
    return c.width > 0 && c.height > 0 && c.width <= GSC_NOALLOC_MAX_SIDE && c.height <= GSC_NOALLOC_MAX_SIDE &&
           c.fovx > 0 && c.fovx < M_PI && c.fovy > 0 && c.fovy < M_PI && c.znear > 0;
}

}  // namespace

}  // namespace gsc

using namespace gsc;

int gsc_render_gaussians_noalloc(const gsc_gaussians* g, const gsc_camera* cam, float* out_chw, float* out_T,
                                 int32_t* status, void* stream) {
    if (!g || !cam || !out_chw) return global_fail(GSC_E_INVALID_ARG, "gsc_render_gaussians_noalloc: null argument");
    if (g->n < 0 || g->n > GSC_NOALLOC_MAX_GAUSSIANS)
        return global_fail(GSC_E_INVALID_ARG, "gsc_render_gaussians_noalloc: n = " + std::to_string(g->n) +
                                                  " outside [0, GSC_NOALLOC_MAX_GAUSSIANS = " +
                                                  std::to_string((long long)GSC_NOALLOC_MAX_GAUSSIANS) + "]");
    if (g->n > 0 && (!g->mu || !g->cov || !g->rgb || !g->alpha))
        return global_fail(GSC_E_INVALID_ARG, "gsc_render_gaussians_noalloc: bad Gaussian arrays");
    if (!na_camera_ok(*cam))
        return global_fail(GSC_E_INVALID_ARG, "gsc_render_gaussians_noalloc: invalid camera or image larger than "
                                              "GSC_NOALLOC_MAX_SIDE");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return global_fail(GSC_E_HIP, std::string("gsc_render_gaussians_noalloc: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kNaDevices) return global_fail(GSC_E_INVALID_ARG, "gsc_render_gaussians_noalloc: device id");
    NaDevice* d = nullptr;
    int rc = na_setup(dev, d);
    if (rc != GSC_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    Raster r = d->r;  // the host-side fields raster_batch updates stay per call
    SegTable tab;
    std::memset(&tab, 0, sizeof(tab));
    tab.n = 1;
    Seg& s = tab.s[0];
    s.L0 = d->L0; s.L1 = d->L1; s.L2 = d->L2; s.L3 = d->L3; s.G = nullptr; s.nG = nullptr;
    s.anchor_pos = nullptr; s.line_anchor = nullptr; s.k = 1;
    s.nG_host = (int32_t)g->n;
    seg_camera(s, *cam);
    s.tile_base = 0;
    s.out_rgb = out_chw; s.out_T = out_T; s.out_nc = nullptr;
    tab.total_tiles = s.ntx * s.nty;
    e = pack_explicit(*g, d->L0, d->L1, d->L2, d->L3, st);
    if (e == hipSuccess) e = raster_batch(tab, r, false, false, st);
    if (e == hipSuccess && status) {
        hipLaunchKernelGGL(k_na_status, dim3(1), dim3(64), 0, st, r.cnt, status);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return global_fail(GSC_E_HIP, std::string("gsc_render_gaussians_noalloc: ") + hipGetErrorString(e));
    return GSC_OK;
}
