// The context object behind the opaque gsc_ctx handle.
#pragma once
#include <string>
#include <vector>

#include "gsc_common.h"

struct gsc_ctx {
    gsc_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    std::vector<void*> allocs;       // device allocations owned by the context
    std::vector<void*> host_allocs;  // pinned host allocations
    std::vector<void*> xallocs;      // buffers of the raster-only entry
    std::vector<void*> xhost_allocs;
    std::vector<void*>* alloc_list = nullptr;  // where dalloc records (nullptr = allocs)
    gsc::Scene scene;
    gsc::View view[2];               // view[1] only without de-redundancy (per-eye derive)
    gsc::Raster raster;
    gsc::Raster xraster;             // raster-only entry
    int nviews = 1;
    bool loaded = false, have_pair = false, derived = false, rendered = false, explicit_render = false;
    gsc_camera eye[2]{}, unified{};
    double t_arrival = 0.0;
    int64_t frame = -1;
    gsc::SegTable last_tab{};
    // explicit Gaussians of the raster-only entry (allocated on first use)
    int64_t xg_cap = 0;
    size_t xg_bytes = 0;
    struct {
        float4* L0;
        float4* L1;
        float4* L2;
        float* L3;
    } xg{};
    // reuse predictor
    float* pred_w = nullptr;      // fp32 parameters
    uint16_t* pred_wbf = nullptr; // bf16 copy for inference
    float* pred_m = nullptr;      // Adam moments
    float* pred_v = nullptr;
    float* pred_g = nullptr;      // gradients
    float* pred_loss = nullptr;   // [1]
    float* pred_X = nullptr;      // training set (device)
    float* pred_y = nullptr;
    int32_t* pred_idx = nullptr;  // batch row order
    int64_t pred_cap = 0;
    int pred_step = 0;
    bool pred_loaded = false;
    int collect_features = 0;
};

namespace gsc {
hipError_t explicit_gaussians(gsc_ctx* c, const gsc_gaussians& g, int64_t ntiles);
void free_explicit(gsc_ctx* c);
void pred_free(gsc_ctx* c);
template <typename T>
hipError_t dalloc(gsc_ctx* c, size_t& acct, T** p, int64_t count);
}  // namespace gsc
