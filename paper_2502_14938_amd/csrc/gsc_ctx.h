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
    float* pred_work = nullptr;   // per-row activations and gradients of a batch
    int32_t* pred_idx = nullptr;
    int pred_step = 0;            // Adam steps taken
    bool pred_loaded = false;
    int collect_features = 0;
    std::vector<void*> pred_allocs;
    // label generation: fresh derivations of the reuse candidates
    float4* lab_L0 = nullptr;
    float4* lab_L1 = nullptr;
    float4* lab_L2 = nullptr;
    float* lab_L3 = nullptr;
    int32_t* lab_iota = nullptr;
    uint8_t* lab_y = nullptr;
};

namespace gsc {
hipError_t explicit_gaussians(gsc_ctx* c, const gsc_gaussians& g, int64_t ntiles);
void free_explicit(gsc_ctx* c);
void pred_free(gsc_ctx* c);

// Device allocation recorded in the context (in *alloc_list when set).
template <typename T>
inline hipError_t dalloc(gsc_ctx* c, size_t& acct, T** p, int64_t count) {
    size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e == hipSuccess) {
        acct += bytes;
        (c->alloc_list ? c->alloc_list : &c->allocs)->push_back((void*)*p);
    }
    return e;
}
}  // namespace gsc
