/*
 * gscache.h -- C ABI of libgscache.so, an MI355X (gfx950) implementation of
 * the per-frame hot path of a cache-centric structured-3DGS stereo renderer
 * (GS-Cache, arXiv 2502.14938).
 *
 * One frame of one viewer is:
 *   gsc_set_camera_pair   unified camera of the stereo pair (Section 4,
 *                         binocular stereo de-redundancy, eqs. 5-6)
 *   gsc_derive            anchor indexing and filtering, cache scheduling
 *                         with dynamic reuse depth, derivation of the misses,
 *                         compose of the render buffer (Section 4, Alg. 1,
 *                         eq. 4; Section 3.1 eq. 3; Section 6 AnchorDecoder)
 *   gsc_render_stereo     per-eye EWA projection, opacity-aware exact tile
 *                         binning, (tile | depth) radix sort, front-to-back
 *                         compositing (Section 3.1; Section 6
 *                         RasterizeGaussians)
 *
 * Conventions for every call:
 *   - Return value: GSC_OK (0) or a negative GSC_E_* code.  No exception or
 *     abort crosses the ABI; gsc_last_error() gives a message.
 *   - "device" pointers are HIP device memory on the context's device
 *     (e.g. a torch CUDA tensor's data_ptr()); "host" pointers are ordinary
 *     process memory.  The library never frees caller memory and never keeps
 *     a caller pointer after a call returns unless stated.
 *   - Work is enqueued on the context's HIP stream (set at creation, NULL =
 *     the legacy default stream) and is asynchronous unless stated; the
 *     caller synchronises that stream (or calls gsc_sync) before reading
 *     outputs.
 *   - A context is used by one host thread at a time.
 */
#ifndef GSCACHE_H
#define GSCACHE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSC_OK 0
#define GSC_E_INVALID_ARG (-1) /* null pointer, size out of range, bad enum */
#define GSC_E_NOT_LOADED (-2)  /* call needs gsc_load_anchors / a camera pair / a derive first */
#define GSC_E_OOM (-3)         /* device allocation failed */
#define GSC_E_CAPACITY (-4)    /* tile-pair or cache capacity exceeded this frame (see stats) */
#define GSC_E_BUDGET (-5)      /* serving: viewer does not fit the HBM budget now */
#define GSC_E_HIP (-6)         /* a HIP runtime call failed */
#define GSC_E_UNCHANGED (-7)   /* serving queue: pose changed less than the threshold; not queued */
#define GSC_E_TIMEOUT (-8)     /* serving queue (poll status): older than the timeout; dropped unrendered */
#define GSC_E_EXPIRED (-9)     /* serving queue (poll status): a newer frame of the viewer was delivered first */

/* Derivation arithmetic (the projection and compositing are always FP32). */
#define GSC_PREC_F32 0  /* FP32 weights, activations and accumulation */
#define GSC_PREC_BF16 1 /* BF16 weights and activations on MFMA, FP32 accumulate */
#define GSC_PREC_FP8 2  /* e4m3fn weights (per-output-row FP32 scale), BF16 activations, FP32 accumulate */

/* Pipeline switches (gsc_config.flags). */
#define GSC_FLAG_DEREDUNDANCY 1u  /* derive once per pair with the unified camera (eqs. 5-6);
                                     off: each eye selects and derives with its own camera */
#define GSC_FLAG_REUSE 2u         /* computation cache across frames (Section 4, Alg. 1) */
#define GSC_FLAG_PREDICTOR 4u     /* learned reuse: cached anchors the predictor marks stale are
                                     re-derived (only adds misses) */
#define GSC_FLAG_FULL_KEY_SORT 8u /* sort full 64-bit (tile<<32 | depth) keys after duplication
                                     instead of pre-sorting depths per Gaussian; same order */
#define GSC_FLAG_LOD_FADE 16u     /* fractional level transition (a reading of the distance-driven
                                     levels of detail of Section 3.1, as in the cited Octree-GS):
                                     an anchor of level l > 0 is selected while its distance to the
                                     unified camera is below 2 d_l (d_l = d_ref 2^-l) and its
                                     Gaussians are rasterised with opacity alpha * w, w =
                                     clamp(2 - dist / d_l, 0, 1): full weight up to d_l, fading to
                                     0 over the next octave of distance.  The cache and the render
                                     buffer's alpha > 0 mask keep the derived alpha. */

/* Cache depth guiding function H (eq. 4). */
#define GSC_GUIDE_LINEAR 0 /* d = clamp(round_half_up(d_max (1 - r)), 1, d_max), r = misses/visible */
#define GSC_GUIDE_FIXED 1  /* d = d_max every frame */
/* Responses for accelerating and for staged motion (Section 7 names them,
 * without formulas; these are integer readings of them): */
#define GSC_GUIDE_EXP 2    /* d = clamp(d_max >> floor(8 r), 1, d_max): halved per eighth of update rate */
#define GSC_GUIDE_STAGED 3 /* d = d_max if r < 1/8, max(1, d_max / 2) if r < 3/8, else 1 */

typedef struct gsc_config {
    int32_t k;                  /* neural Gaussians per anchor (offsets), 1..16 */
    int32_t feat_dim;           /* anchor feature length F, must be 32 */
    int32_t hidden;             /* MLP hidden width, must be 32 */
    int32_t d_max;              /* maximum reuse depth D_max (the paper uses 10), 1..64 */
    int32_t guide;              /* GSC_GUIDE_* */
    int32_t precision;          /* GSC_PREC_* */
    uint32_t flags;             /* GSC_FLAG_* */
    float predictor_threshold;  /* re-derive when p(stale) > this */
    int64_t cache_capacity;     /* cache lines (anchors); 0 = number of anchors */
    int32_t max_width;          /* largest eye image the context renders */
    int32_t max_height;
    int64_t max_pairs;          /* tile-pair capacity per eye; 0 = 24 x max Gaussians */
} gsc_config;

/* Pinhole camera: world -> camera rotation R (row-major 3x3, rows = right,
 * down, forward), centre pos, full fields of view (radians), image size,
 * near plane.  Pixel (u, v) has its centre at (u + 0.5, v + 0.5);
 * fx = width / (2 tan(fovx / 2)), principal point (width/2, height/2). */
typedef struct gsc_camera {
    double R[9];
    double pos[3];
    double fovx, fovy;
    int32_t width, height;
    double znear;
} gsc_camera;

/* Anchor scene (Section 3.1: anchors with feature f, derived by MLP_theta).
 * All arrays are row-major float32 (level uint8) in host memory
 * (is_device = 0) or device memory (is_device = 1):
 *   pos [n,3], level [n], radius [n] (bounding sphere of everything the
 *   anchor derives), feat [n,F], scale [n,6] ([0:3] offset scale, [3:6]
 *   base Gaussian scale), offsets [n,k,3].
 * d_ref: LOD reference distance; an anchor of level l > 0 is used only
 * within d_ref * 2^-l of the unified camera (2 d_ref 2^-l with
 * GSC_FLAG_LOD_FADE).
 * dist_unit: 0, or > 0 for MLPs that take the anchor's distance to the
 * unified camera as an input after the view direction (the cited methods'
 * optional camera-distance feature): layer 1 then reads [f; d_view;
 * |x - p_u| / dist_unit] and W1[h] has F + 4 columns (see gsc_mlp). */
typedef struct gsc_anchors {
    int64_t n;
    const float* pos;
    const uint8_t* level;
    const float* radius;
    const float* feat;
    const float* scale;
    const float* offsets;
    double d_ref;
    int32_t is_device;
    double dist_unit;
} gsc_anchors;

/* Derivation MLPs (eq. 3), host float32, row-major [out, in] like
 * torch.nn.Linear; head 0 = opacity (k outputs), 1 = colour (3k), 2 =
 * covariance (7k: 3 scale logits then quaternion w,x,y,z per Gaussian).
 * W1[h] is [hidden, F+3] (inputs: feature then view direction), or
 * [hidden, F+4] when gsc_anchors.dist_unit > 0 (then the scaled distance),
 * W2[h] is [c_h k, hidden]. */
typedef struct gsc_mlp {
    const float* W1[3];
    const float* b1[3];
    const float* W2[3];
    const float* b2[3];
} gsc_mlp;

/* Explicit Gaussians for the raster-only entry, device float32:
 * mu [n,3], cov [n,6] (xx xy xz yy yz zz), rgb [n,3], alpha [n]. */
typedef struct gsc_gaussians {
    int64_t n;
    const float* mu;
    const float* cov;
    const float* rgb;
    const float* alpha;
} gsc_gaussians;

/* Per-frame counters, valid after gsc_sync. */
typedef struct gsc_frame_stats {
    int64_t frame;          /* frame index t of the last derive */
    int64_t n_visible;      /* |X_t| */
    int64_t n_miss;         /* |M_t| anchors derived this frame */
    int64_t n_gauss;        /* |G_t| Gaussians in the render buffer */
    int64_t n_pairs[2];     /* tile pairs per eye */
    int64_t n_evicted;      /* lines evicted for capacity this frame */
    int32_t depth_used;     /* reuse depth d_t applied this frame */
    int32_t depth_next;     /* d_{t+1} */
    int32_t overflow;       /* bit0 raster capacity (tile pairs, entries, tall-row spans), bit1 cache capacity */
    int32_t pad;
    int64_t device_bytes;   /* device memory owned by the context */
    int64_t n_eval[2];      /* (pixel, Gaussian) visits of the blend per eye: per
                               pixel, the Gaussians visited front to back until
                               its transmittance ran out or its list ended
                               (0 unless gsc_count_work is on) */
    int64_t n_contrib[2];   /* of those, the visits that were composited */
    int64_t n_tall;         /* Gaussians (both eyes) whose footprint spans more than 4 tile rows */
} gsc_frame_stats;

typedef struct gsc_ctx gsc_ctx;

/* Create a context on the current HIP device.  cfg is copied; stream is a
 * hipStream_t (NULL = default stream).  *out receives the context. */
int gsc_create(const gsc_config* cfg, void* stream, gsc_ctx** out);
/* Free the context and every device buffer it owns (synchronises first). */
void gsc_destroy(gsc_ctx* ctx);
/* Message for the last error on this context (or a global one if ctx is
 * NULL); valid until the next call. */
const char* gsc_last_error(const gsc_ctx* ctx);
/* Change the stream later calls enqueue on. */
int gsc_set_stream(gsc_ctx* ctx, void* stream);

/* Copy the scene and MLP weights into the library's own device layout (SoA
 * positions, packed weights in every precision), then synchronise: the
 * caller may free its arrays on return.  Resets the cache and frame count. */
int gsc_load_anchors(gsc_ctx* ctx, const gsc_anchors* anchors, const gsc_mlp* mlp);

/* Set the next frame's stereo pair (host structs, copied).  Both eyes must
 * share fov, size and near plane; size must fit max_width x max_height.
 * Computes the unified camera in FP64 on the host (eqs. 5-6; roll from the
 * mean of the eyes' right axes).  t_arrival is recorded for latency stats. */
int gsc_set_camera_pair(gsc_ctx* ctx, const gsc_camera* left, const gsc_camera* right, double t_arrival);

/* Enqueue anchor selection, cache scheduling (+ learned reuse), derivation
 * of the misses, depth update and compose for frame t, then t += 1.
 * Needs gsc_load_anchors and gsc_set_camera_pair. */
int gsc_derive(gsc_ctx* ctx);

/* Enqueue rasterisation of the composed render buffer for both eyes into
 * caller-owned device buffers: rgb planar [3,H,W] float32 per eye; final
 * transmittance [H,W] float32 per eye (may be NULL).  Needs gsc_derive. */
int gsc_render_stereo(gsc_ctx* ctx, float* left_chw, float* right_chw, float* left_T, float* right_T);

/* Raster-only entry: rasterise explicit Gaussians (device arrays) for one
 * camera into out_chw [3,H,W] float32, out_T [H,W] (may be NULL) and
 * out_ncontrib [H,W] int32 (may be NULL).  n must not exceed the context's
 * Gaussian capacity.  Does not touch the cache. */
int gsc_render_gaussians(gsc_ctx* ctx, const gsc_gaussians* g, const gsc_camera* cam, float* out_chw,
                         float* out_T, int32_t* out_ncontrib);

/* Allocation-free variant of gsc_render_gaussians, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  No context: the intermediate buffers
 * (the Gaussians' staged copy, per-Gaussian records, sort keys, tile pairs,
 * ranges, counters) live in one static device array of the library (48 MiB,
 * held by each device that loads the library until the process ends), and
 * the call allocates nothing.  Same kernels and results as
 * gsc_render_gaussians (depth pre-sorted pairs, no work counting).
 * g: device arrays as for gsc_render_gaussians, n <= GSC_NOALLOC_MAX_GAUSSIANS;
 * cam: host, width and height <= GSC_NOALLOC_MAX_SIDE; out_chw [3,H,W] and
 * out_T [H,W] (may be NULL): caller-owned device float32; status (device,
 * may be NULL) receives the overflow bits after the kernels run (0, or bit0
 * when more than GSC_NOALLOC_MAX_PAIRS tile pairs were needed and the excess
 * dropped).  stream: hipStream_t (NULL = default stream); asynchronous.
 * Sizes beyond the maxima return GSC_E_INVALID_ARG before any device work.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (other streams, other host threads) race. */
#define GSC_NOALLOC_MAX_GAUSSIANS 65536
#define GSC_NOALLOC_MAX_PAIRS (1 << 21)
#define GSC_NOALLOC_MAX_SIDE 2048
int gsc_render_gaussians_noalloc(const gsc_gaussians* g, const gsc_camera* cam, float* out_chw, float* out_T,
                                 int32_t* status, void* stream);

/* Wait for the stream, then report GSC_E_CAPACITY if the last frame
 * overflowed a capacity, else GSC_OK. */
int gsc_sync(gsc_ctx* ctx);
/* Synchronise and fill *st with the last frame's counters. */
int gsc_get_stats(gsc_ctx* ctx, gsc_frame_stats* st);
/* Drop every cache line and reset the depth to d_max and t to 0. */
int gsc_reset_cache(gsc_ctx* ctx);

/* Debug copies for parity tests (synchronous).  what: */
#define GSC_DBG_VISIBLE 0   /* int32 [n_visible] anchor ids, ascending */
#define GSC_DBG_MISSES 1    /* int32 [n_miss] anchor ids, ascending */
#define GSC_DBG_GAUSS 2     /* int32 [n_gauss] (visible position * k + j) of the render buffer */
#define GSC_DBG_DERIVED 3   /* float32 [n_gauss, 13]: mu3 cov6 rgb3 alpha, render-buffer order */
#define GSC_DBG_PAIRS 4     /* int32 [n_pairs(eye), 2]: (tile, render-buffer index), each tile's
                               depth-ordered list as the blend reads it, tiles in order */
#define GSC_DBG_RANGES 5    /* int32 [n_tiles(eye), 2]: [start, end) of each tile's list in the above */
#define GSC_DBG_PREPROC 6   /* float32 [n_gauss, 8]: mean2d.x, .y, conic a b c, alpha, depth,
                               tile count (as float) for eye */
#define GSC_DBG_DEPTH 7     /* int32 [1]: current reuse depth */
#define GSC_DBG_SORT_KEYS 8 /* uint32 [sorted items of the last raster batch]: the sorted keys, global
                               super-tile ids (a super tile is 2x2 tiles; images in order), as the
                               ranges read them */
#define GSC_DBG_RAW_RANGES 9 /* int32 [global super tiles, 2]: [start, end) of every super tile in the
                               sorted keys ([0, 0) for one without pairs) */
#define GSC_DBG_SORT_VALS 10 /* uint32 [sorted items]: entry | mask << 28, the mask's bit
                               2 (ty & 1) + (tx & 1) set for each tile of the super tile the entry's
                               footprint covers; a tile's list (GSC_DBG_PAIRS) is its super tile's
                               list filtered by its bit */
/* Copies at most cap elements (of the unit above: ints, floats or rows) to
 * host_dst and writes the full count to *n. */
int gsc_debug_copy(gsc_ctx* ctx, int what, int eye, void* host_dst, int64_t cap, int64_t* n);

/* With enable != 0 the blend of later frames also counts its work per eye
 * (gsc_frame_stats n_eval, n_contrib); off by default, since the counters
 * cost the blend a few instructions per (pixel, Gaussian) visit.  The
 * raster-only entry counts whenever it is asked for per-pixel counts. */
int gsc_count_work(gsc_ctx* ctx, int enable);

/* Two frames in flight (enable != 0): each stereo frame's blend runs on a
 * stream the library owns, overlapping the next frame's selection, schedule,
 * derivation, composition, preprocess, sorts and emission on the context's
 * stream.  Frames alternate between two raster buffer sets (the second one
 * is allocated here, once per loaded scene, the size of the first), and a
 * frame reuses a set only after the blend that last read it has finished.
 * A frame's output images are complete only after gsc_sync (or another call
 * documented to wait for the stream); the caller must not read them, or
 * reuse their memory, before.  The images are those of the sequential order
 * (same kernels, same inputs).  Waits for the streams; requires a loaded
 * scene to enable (GSC_E_NOT_LOADED); GSC_E_OOM if the second set does not
 * fit.  Off by default; loading a scene switches it off.  Section 5 renders
 * whole frames asynchronously on several GPU workers; on one GPU this
 * overlaps the stages of consecutive frames instead. */
int gsc_pipeline(gsc_ctx* ctx, int enable);

/* Mean SSIM of two device images a, b (float32 [channels, height, width],
 * values in [0, 1]) into *out (host): the quality table's third metric
 * (Table 4), as Wang et al. define it: an 11 x 11 Gaussian window (sigma
 * 1.5, normalised), C1 = 0.01^2, C2 = 0.03^2, the map averaged over every
 * window position inside the image and over channels.  Waits for the
 * context's streams first (the images may come from a frame in flight) and
 * at the end; allocates a small scratch buffer per call.  height and width
 * at least 11, channels 1..65535 (GSC_E_INVALID_ARG otherwise). */
int gsc_ssim(gsc_ctx* ctx, const float* a, const float* b, int32_t channels, int32_t height, int32_t width,
             double* out);

/* ---------------- stage timing -------------------------------------------
 * With timing on, every frame (gsc_derive + gsc_render_stereo) records HIP
 * events on the context's stream at its stage boundaries; gsc_timing_read
 * synchronises and returns the summed device milliseconds per stage over the
 * frames issued since timing was switched on or last read.  Stages: */
#define GSC_STAGE_SCHEDULE 0    /* unified-camera selection, cache schedule */
#define GSC_STAGE_DERIVE 1      /* MLP derivation of the misses (MFMA) */
#define GSC_STAGE_COMPOSE 2     /* depth update, render buffer */
#define GSC_STAGE_PREPROCESS 3  /* projection, conic, extent, spans of footprints up to 4 tile rows */
#define GSC_STAGE_TALL_SPANS 4  /* row spans and tile counts of taller footprints */
#define GSC_STAGE_DEPTH_SORT 5  /* per-Gaussian depth radix passes */
#define GSC_STAGE_PAIR_SCAN 6   /* pair offsets in depth order */
#define GSC_STAGE_DUP_ROWS 7    /* pair emission, footprints of up to 4 tile rows */
#define GSC_STAGE_TALL_LIST 8   /* dense list of the taller footprints */
#define GSC_STAGE_DUP_BIG 9     /* pair emission, taller footprints */
#define GSC_STAGE_TILE_SORT 10  /* tile-id radix passes over the pairs */
#define GSC_STAGE_RANGES 11     /* per-tile ranges */
#define GSC_STAGE_BLEND 12      /* blend */
#define GSC_NUM_STAGES 13
/* Switch timing on (enable != 0) or off; clears what was recorded.  Waits
 * for the stream. */
int gsc_timing(gsc_ctx* ctx, int enable);
/* ms_out host [n] (n <= GSC_NUM_STAGES): summed ms per stage; frame_ms host
 * [frame_cap] (may be NULL when frame_cap is 0): each recorded frame's device
 * time from the start of its derive stage to the end of its blend (-1 when
 * the frame did not run both); *frames = frames recorded.  The events skip
 * the system-scope fence (no cache writeback per mark).  Clears the record. */
int gsc_timing_read(gsc_ctx* ctx, double* ms_out, int32_t n, double* frame_ms, int64_t frame_cap, int64_t* frames);
/* Which stages get boundary events while timing is on: bit i of stage_mask
 * selects stage i (default: all).  The frame's first and last events are
 * always recorded.  Each event makes the stream wait for the kernel before it
 * to drain (a few microseconds), so timing a few stages disturbs the frame
 * less than timing all; stages not selected read 0. */
int gsc_timing_stages(gsc_ctx* ctx, uint32_t stage_mask);

/* ---------------- learned reuse predictor (Linear 6-64-64-1, sigmoid) ----
 * An extension of the reuse decision of Section 4 (Alg. 1): for a
 * visible anchor whose cache line is still valid, a small MLP reads six
 * features (view-direction change, distance ratio, age / d_max, level /
 * l_max, camera travel / distance, log2 projected voxel size) and predicts
 * whether reusing it would visibly change its Gaussians; with
 * GSC_FLAG_PREDICTOR set, anchors with p > predictor_threshold are derived
 * again (the predictor only adds misses).  Inference uses BF16 weights and
 * activations with FP32 accumulation. */
#define GSC_PRED_NPARAMS (64 * 6 + 64 + 64 * 64 + 64 + 64 + 1)
/* Load predictor parameters (host float32 [GSC_PRED_NPARAMS], order W1[64,6]
 * b1[64] W2[64,64] b2[64] W3[1,64] b3[1], rows = outputs). */
int gsc_predictor_load(gsc_ctx* ctx, const float* params, int64_t n);
/* Copy the current parameters to host float32 [GSC_PRED_NPARAMS]. */
int gsc_predictor_get(gsc_ctx* ctx, float* params, int64_t n);
/* Record the reuse candidates (visible anchors holding a valid line) and
 * their features during later gsc_derive calls (enable != 0) or stop. */
int gsc_predictor_collect(gsc_ctx* ctx, int enable);
/* Training data from the last gsc_derive (collection on, predictor off):
 * every candidate anchor is derived again with this frame's unified camera
 * in FP32 and compared with its cached Gaussians.  A Gaussian's drift is
 * the largest of |d opacity|, opacity * |d colour| (any channel) and
 * opacity * (max |d cov| / max |cov|) / 2; label 1 (re-derive) iff the
 * anchor's largest drift times its projected footprint area in pixels,
 * max(1, size^2) with size = 2^X[5], exceeds 16/255 (one 8-bit level over a
 * 4x4-pixel patch).  Collect with the predictor off.  Writes up to cap rows:
 * X_out host float32 [cap, 6], y_out host uint8 [cap], ids_out host int32
 * [cap] anchor ids (may be NULL); *n = candidate count.  Synchronous. */
int gsc_predictor_labels(gsc_ctx* ctx, float* X_out, uint8_t* y_out, int32_t* ids_out, int64_t cap, int64_t* n);
/* Train on the device with the library's own forward, backward and Adam
 * kernels: X host float32 [n,6], y host uint8 [n].  Mini-batches of `batch`
 * rows (<= 4096) in a shuffled order seeded by `seed`, for `epochs` epochs;
 * mean BCE with positive-class weight pos_weight; Adam(lr, 0.9, 0.999,
 * 1e-8).  loss_out (host, may be NULL) receives each epoch's mean loss.
 * Synchronous. */
int gsc_predictor_train(gsc_ctx* ctx, const float* X, const uint8_t* y, int64_t n, int32_t batch,
                        int32_t epochs, float lr, float pos_weight, uint64_t seed, float* loss_out);
/* One forward/backward pass over device arrays X [n,6] float32 and y [n]
 * float32 (0/1), n <= 4096: mean loss and gradients (host float32
 * [GSC_PRED_NPARAMS]), FP32.  Synchronous. */
int gsc_predictor_grad(gsc_ctx* ctx, const float* X, const float* y, int64_t n, float pos_weight,
                       float* grads_out, float* loss_out);
/* p(stale) for device X [n,6] into device p_out [n] (BF16 inference path). */
int gsc_predictor_infer(gsc_ctx* ctx, const float* X, int64_t n, float* p_out);

/* ---------------- serving: several viewers, one device -------------------
 * An extension around the per-frame path of Section 4 (the paper's
 * own scheduler, Section 5, is multi-GPU and not this): continuous batching
 * of stereo frame requests from several viewers of uneven resolution, each
 * with its own device cache, over one shared scene.  Every call on a server
 * comes from one host thread; calls on one server never overlap. */
typedef struct gsc_server gsc_server;
/* A server shares the scene (and predictor) of `scene_ctx`, which must stay
 * alive, be loaded with de-redundancy on, and not be rendered with while the
 * server runs.  budget_bytes caps the device memory of all admitted viewers
 * (their caches, per-frame buffers and batch-raster shares).  All work goes
 * on `stream` (NULL = the default stream). */
int gsc_server_create(gsc_ctx* scene_ctx, int64_t budget_bytes, void* stream, gsc_server** out);
/* Waits for outstanding batches, then frees everything. */
void gsc_server_destroy(gsc_server* s);
const char* gsc_server_last_error(const gsc_server* s);
/* Device bytes a viewer of at most max_width x max_height per eye takes:
 * cache lines (capacity of the scene context's config, or one per anchor),
 * slot map, per-frame lists, and its share of the batch raster (entries for
 * two eyes of a full cache, tile pairs: max_pairs of the config, else
 * 16 per pixel of both eyes within [2^22, min(24 per entry, 2^27)]). */
int64_t gsc_server_viewer_bytes(gsc_server* s, int32_t max_width, int32_t max_height);
/* Admit a viewer: returns a viewer id >= 0, or GSC_E_BUDGET when its bytes
 * do not fit the budget beside the viewers already admitted (retry after
 * one leaves).  Waits for outstanding batches (the batch raster is resized). */
int gsc_server_admit(gsc_server* s, int32_t max_width, int32_t max_height);
/* Queue one stereo frame for a viewer: cameras are copied (eyes share
 * intrinsics, at most the admitted size); outputs are caller device buffers
 * float32 [3,H,W] per eye that must stay valid until the request completes.
 * t_arrival is carried for FIFO order.  Returns a request id >= 0. */
int64_t gsc_server_submit(gsc_server* s, int32_t viewer, const gsc_camera* left, const gsc_camera* right,
                          double t_arrival, float* out_left, float* out_right);
/* Form one batch from the oldest queued request of each of up to 8 viewers
 * (oldest arrival first) and enqueue it: per viewer the derive stage on its
 * own cache, then one raster batch over all (viewer, eye) images, ending in
 * one blend launch over every (viewer, eye, tile).  Asynchronous; returns
 * the number of requests launched (0 when nothing is queued).  If enqueuing
 * fails (GSC_E_HIP), the requests taken for the batch complete at once with
 * status GSC_E_HIP. */
int gsc_server_step(gsc_server* s);
/* Completed requests since the last poll (non-blocking): writes up to cap
 * request ids, completion times (seconds on the host monotonic clock, taken
 * when the device finished the batch) and statuses (GSC_OK, or
 * GSC_E_CAPACITY when the batch ran out of cache lines or tile pairs; status
 * may be NULL); returns the count. */
int gsc_server_poll(gsc_server* s, int64_t* ids, double* t_done, int32_t* status, int32_t cap);
/* Requests queued or in flight. */
int gsc_server_pending(gsc_server* s);
/* Queue policy of Section 5 (each part off when its argument is negative or
 * zero; all off by default):
 *   pose gate: gsc_server_submit queues a request only when its unified
 *     camera moved more than pose_m (metres) or turned more than pose_rad
 *     (radians, angle between viewing directions) since the viewer's last
 *     queued request; otherwise it returns GSC_E_UNCHANGED, nothing queued;
 *   timeout: gsc_server_step drops queued requests whose t_arrival is more
 *     than timeout_s before the host monotonic clock (t_arrival must be on
 *     that clock), unrendered; poll reports them with GSC_E_TIMEOUT;
 *   ordered (nonzero): a request that finishes after a request of the same
 *     viewer with a later t_arrival was delivered is discarded; poll reports
 *     it with GSC_E_EXPIRED (its output buffers hold the render anyway).
 * Applies to later calls; queued requests keep their place. */
int gsc_server_policy(gsc_server* s, double pose_m, double pose_rad, double timeout_s, int ordered);
/* Two batches in flight (Section 5's asynchronous rendering of whole frames,
 * on one GPU): with enable nonzero, a batch's blend runs on a stream of its
 * own while the next batch's derive stages (selection, cache schedule,
 * derivation, compose) and raster stages up to the tile ranges run on the
 * server's stream, so a request that arrives while a batch is on the GPU
 * starts its work beside that batch's blend.  Two raster buffer sets
 * alternate by batch, so each admitted viewer counts its raster share twice
 * against the budget.  Images are the same as with one batch at a time.
 * Must be called before any viewer is admitted (else GSC_E_INVALID_ARG);
 * synchronises the server's streams. */
int gsc_server_overlap(gsc_server* s, int enable);
/* Remove a viewer with no queued requests and free its buffers (waits for
 * outstanding batches). */
int gsc_server_leave(gsc_server* s, int32_t viewer);

#ifdef __cplusplus
}
#endif
#endif /* GSCACHE_H */
