// The context object behind the opaque gsc_ctx handle.
#pragma once
#include <string>
#include <vector>

#include "gsc_common.h"

namespace gsc {
// Device and pinned host allocations owned together (freed together).
struct AllocSet {
    std::vector<void*> dev, host;
    size_t bytes = 0;  // device bytes
    void release() {
        for (void* p : dev) (void)hipFree(p);
        for (void* p : host) (void)hipHostFree(p);
        dev.clear();
        host.clear();
        bytes = 0;
    }
    bool empty() const { return dev.empty() && host.empty(); }
};

// Device allocation of count elements recorded in `set`; acct also counts it.
template <typename T>
inline hipError_t dalloc(AllocSet& set, size_t& acct, T** p, int64_t count) {
    size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e == hipSuccess) {
        acct += bytes;
        set.bytes += bytes;
        set.dev.push_back((void*)*p);
    }
    return e;
}

template <typename T>
inline hipError_t halloc(AllocSet& set, T** p, int64_t count) {
    hipError_t e = hipHostMalloc((void**)p, (size_t)(count > 0 ? count : 1) * sizeof(T));
    if (e == hipSuccess) set.host.push_back((void*)*p);
    return e;
}

// Buffers of one raster batch.
template <class Fn>
hipError_t raster_layout(Raster& r, int64_t max_entries, int64_t max_pairs, int64_t max_tiles, bool full_key, Fn&& A) {
    hipError_t e;
#define A_(p, cnt) if ((e = A(p, cnt)) != hipSuccess) return e
    A_(r.rec, 4 * max_entries); A_(r.ntiles, max_entries); A_(r.nsup, max_entries); A_(r.scnt, max_entries);
    A_(r.pt_list, max_entries); A_(r.pt_pack, max_entries / 256 + 1); A_(r.pt_off, max_entries / 256 + 1);
    // tall footprints: at most a quarter of the entries (more are flagged as overflow)
    A_(r.trec, max_entries / 4 + 256); A_(r.pt_sroff, max_entries / 4 + 256);
    A_(r.srow, max_entries); A_(r.srow_y, max_entries);
    A_(r.dkey[0], max_entries); A_(r.dkey[1], max_entries);
    A_(r.dval[0], max_entries); A_(r.dval[1], max_entries); A_(r.offs, max_entries);
    A_(r.pkey[0], max_pairs); A_(r.pkey[1], max_pairs); A_(r.pval[0], max_pairs); A_(r.pval[1], max_pairs);
    if (full_key) { A_(r.pkey64[0], max_pairs); A_(r.pkey64[1], max_pairs); }
    A_(r.ranges, 2 * max_tiles); A_(r.tile_eval, 2 * max_tiles); A_(r.hist, 256 * kSortBlocks);
    A_(r.block_sums, kScanBlocks); A_(r.block_sums64, kScanBlocks);
    A_(r.n_sort, 1); A_(r.cnt, 1);
#undef A_
    return hipSuccess;
}

// Explicit Gaussians (public arrays) into the four line arrays, on st.
hipError_t pack_explicit(const gsc_gaussians& g, float4* L0, float4* L1, float4* L2, float* L3, hipStream_t st);
// Set the thread's context-free error message (gsc_last_error(NULL)).
int global_fail(int code, const std::string& msg);

// Exact device bytes alloc_view / alloc_raster will take (admission planning).
size_t view_bytes(int64_t n, int64_t C, int k);
size_t raster_bytes(int64_t max_entries, int64_t max_pairs, int64_t max_tiles, bool full_key);
hipError_t alloc_view(AllocSet& set, View& v, int64_t n, int64_t C, int k);
hipError_t alloc_raster(AllocSet& set, Raster& r, int64_t max_entries, int64_t max_pairs, int64_t max_tiles,
                        bool full_key);
hipError_t reset_view(View& v, int64_t n, int dmax, hipStream_t st);
DeriveCam derive_cam(const gsc_camera& c, float d_ref, bool fade);
// The fractional level transition's inputs for a segment: the scene's levels
// and d_ref, and the centre of the camera the view derives with.
void seg_lod_fade(Seg& s, const Scene& sc, const gsc_camera& derive_camera);
void unified_camera(const gsc_camera& l, const gsc_camera& r, gsc_camera& u);
bool valid_camera(const gsc_camera& c);
}  // namespace gsc

struct gsc_ctx {
    gsc_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    gsc::AllocSet mem;               // scene, views and raster of the stereo path
    gsc::AllocSet xmem;              // buffers of the raster-only entry
    gsc::AllocSet pmem;              // reuse predictor parameters and training buffers
    gsc::AllocSet lmem;              // label scratch, sized for the loaded scene
    gsc::Scene scene;
    gsc::View view[2];               // view[1] only without de-redundancy (per-eye derive)
    gsc::Raster raster;
    gsc::Raster xraster;             // raster-only entry
    // two frames in flight (gsc_pipeline): a frame's blend runs on
    // blend_stream while the next frame's stages up to its tile ranges run on
    // `stream`; the frames alternate between raster and raster2, and a frame
    // reuses a set only after the blend that last read it has finished
    bool pipeline = false;
    gsc::Raster raster2;
    hipStream_t blend_stream = nullptr;
    hipEvent_t front_done[2] = {nullptr, nullptr};
    hipEvent_t blend_done[2] = {nullptr, nullptr};
    bool blend_pending[2] = {false, false};
    int64_t pipe_frames = 0;
    int last_set = 0;                // raster set of the last stereo frame
    int64_t rcap_entries = 0, rcap_pairs = 0, rcap_tiles = 0;  // raster capacities of the loaded scene
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
    // label generation: fresh derivations of the reuse candidates
    float4* lab_L0 = nullptr;
    float4* lab_L1 = nullptr;
    float4* lab_L2 = nullptr;
    float* lab_L3 = nullptr;
    int32_t* lab_iota = nullptr;
    uint8_t* lab_y = nullptr;
    int64_t lab_entries = 0;      // anchors * k the label scratch holds
    bool count_work = false;       // blend counts visits / contributions (gsc_count_work)
    bool last_count_work = false;  // ... for the last rendered frame
    // stage timing (gsc_timing): one event set per frame since the last read
    bool timing = false;
    uint32_t timing_mask = ~0u;    // stages with boundary events (gsc_timing_stages)
    std::vector<gsc::Marks> marks;
    size_t marks_used = 0;
};

namespace gsc {
// Waits for the context's stream and, with two frames in flight, for the
// blend stream.
hipError_t sync_all(gsc_ctx* c);
hipError_t explicit_gaussians(gsc_ctx* c, const gsc_gaussians& g, int64_t ntiles);
void free_explicit(gsc_ctx* c);
void free_labels(gsc_ctx* c);
void pred_free(gsc_ctx* c);
Marks* frame_marks(gsc_ctx* c);
void free_marks(gsc_ctx* c);
}  // namespace gsc
