// Multi-viewer serving on one device: continuous batching of stereo frame
// requests from several viewers (uneven resolutions, one device cache each)
// over the shared scene of a context.
//
//   admit    a viewer is admitted when its cache, per-frame buffers and its
//            share of the batch raster fit the device-memory budget
//   submit   a frame request is queued on its viewer (cameras copied, the
//            unified camera of eqs. 5-6 computed on the host)
//   step     the oldest queued request of up to kMaxSeg/2 viewers (oldest
//            first) form one batch: each viewer's derive stage (selection,
//            cache schedule, derivation of misses, compose) on its own cache,
//            then ONE raster batch over all (viewer, eye) images, ending in
//            one blend launch over every (viewer, eye, tile); the host
//            returns at once and the next step can be queued behind this one
//   overlap  two batches in flight: a batch's blend runs on a stream of its
//            own while the next batch's derive stages and raster front run
//            on the server's stream, over two raster buffer sets that
//            alternate by batch (a set is reused once the blend that last
//            read it has finished)
//   poll     completions, timestamped on the host monotonic clock by a host
//            function the stream runs when the batch's kernels are done
#include <algorithm>
#include <cmath>
#include <cstring>
#include <ctime>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gsc_common.h"
#include "gsc_ctx.h"

using namespace gsc;

namespace {

constexpr int kMaxBatchViewers = kMaxSeg / 2;
constexpr int64_t kPairCapPerViewer = (int64_t)1 << 27;

double now_monotonic() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct Request {
    int64_t id;
    gsc_camera eye[2];
    gsc_camera unified;
    double t_arrival;
    float* out[2];
};

struct Viewer {
    int32_t max_w = 0, max_h = 0;
    bool has_pose = false;            // pose of the last queued request (pose gate)
    double pose[3] = {0, 0, 0}, dir[3] = {0, 0, 1};
    View v;
    AllocSet mem;
    int64_t entries = 0, pairs = 0, tiles = 0;  // share of the batch raster
    size_t bytes = 0;                           // view + raster share (upper bound)
    std::deque<Request> queue;
};

// Counters a finished batch reports to the host (pinned, one per batch).
struct BatchReport {
    RasterCounters rc;
    Counters vc[kMaxBatchViewers];
};

struct Batch;

}  // namespace

struct gsc_server {
    gsc_ctx* ctx = nullptr;
    hipStream_t st = nullptr;
    int64_t budget = 0;
    size_t used = 0;
    std::vector<std::unique_ptr<Viewer>> viewers;
    AllocSet rmem;
    Raster raster;
    int64_t r_entries = 0, r_pairs = 0, r_tiles = 0;
    int64_t next_id = 0;
    std::string err;
    std::mutex mu;  // guards the fields below (host functions run on a runtime thread)
    struct Done {
        int64_t id;
        double t;
        int32_t status;
    };
    std::vector<Done> done;
    std::vector<double> last_delivered;  // per viewer slot: t_arrival of its last delivered frame
    // queue policy (gsc_server_policy); <= 0: off
    double pose_m = 0.0, pose_rad = 0.0, timeout_s = 0.0;
    bool ordered = false;
    std::vector<BatchReport*> free_reports;
    std::vector<BatchReport*> all_reports;
    int64_t in_flight = 0;
    // two batches in flight (gsc_server_overlap)
    bool overlap = false;
    hipStream_t blend_st = nullptr;
    hipEvent_t front_done[2] = {nullptr, nullptr};
    hipEvent_t blend_done[2] = {nullptr, nullptr};
    hipEvent_t copies_done[2] = {nullptr, nullptr};
    bool blend_pending[2] = {false, false};
    AllocSet rmem2;
    Raster raster2;
    int64_t nbatch = 0;
};

namespace {

struct Batch {
    gsc_server* s;
    BatchReport* rep;
    int nviewers;
    std::vector<int64_t> ids;
    std::vector<int> viewer_of;  // batch-local viewer index of each request
    std::vector<int32_t> viewer_id;
    std::vector<double> t_arrival;
};

int sfail(gsc_server* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

// A batch that failed to enqueue: the requests already taken off their
// viewers' queues complete at once with GSC_E_HIP (so a caller polling for
// them is answered), and the report goes back to the free list.
int abort_batch(gsc_server* s, Batch* b, const std::string& msg) {
    const double t = now_monotonic();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (int64_t id : b->ids) s->done.push_back({id, t, GSC_E_HIP});
        s->free_reports.push_back(b->rep);
    }
    delete b;
    return sfail(s, GSC_E_HIP, msg);
}

void on_batch_done(void* p) {
    Batch* b = (Batch*)p;
    const double t = now_monotonic();
    gsc_server* s = b->s;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const bool pairs_over = (b->rep->rc.overflow & 7) != 0;
        for (size_t i = 0; i < b->ids.size(); ++i) {
            const bool cache_over = (b->rep->vc[b->viewer_of[i]].overflow & 2) != 0;
            int32_t status = (pairs_over || cache_over) ? GSC_E_CAPACITY : GSC_OK;
            if (s->ordered && status == GSC_OK) {
                // display order: never deliver a frame older than one already delivered
                double& last = s->last_delivered[(size_t)b->viewer_id[i]];
                if (b->t_arrival[i] < last) status = GSC_E_EXPIRED;
                else last = b->t_arrival[i];
            }
            s->done.push_back({b->ids[i], t, status});
        }
        s->free_reports.push_back(b->rep);
        s->in_flight -= 1;
    }
    delete b;
}

int64_t viewer_cache_lines(const gsc_ctx* c) {
    const int64_t n = c->scene.n;
    int64_t C = c->cfg.cache_capacity > 0 ? c->cfg.cache_capacity : n;
    if (!(c->cfg.flags & GSC_FLAG_REUSE) && C < n) C = n;  // no-cache schedule: line i = visible i
    return C;
}

void viewer_share(const gsc_ctx* c, int32_t W, int32_t H, int64_t& entries, int64_t& pairs, int64_t& tiles) {
    const int64_t C = viewer_cache_lines(c);
    entries = 2 * C * c->scene.k;
    const int64_t ntx = (W + kTile - 1) / kTile, nty = (H + kTile - 1) / kTile;
    tiles = 2 * ntx * nty;
    if (c->cfg.max_pairs > 0) {
        pairs = c->cfg.max_pairs;
    } else {
        pairs = std::max<int64_t>((int64_t)1 << 22, (int64_t)16 * 2 * W * H);
        pairs = std::min(pairs, std::min<int64_t>(24 * entries, kPairCapPerViewer));
    }
}

// raster_sets: 2 with two batches in flight (each viewer holds a share of both)
size_t viewer_bytes_of(const gsc_ctx* c, int32_t W, int32_t H, int raster_sets) {
    int64_t e, p, t;
    viewer_share(c, W, H, e, p, t);
    return view_bytes(c->scene.n, viewer_cache_lines(c), c->scene.k) + sizeof(Counters) +
           (size_t)raster_sets * raster_bytes(e, p, t, (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0);
}

// Wait for everything the server enqueued (both streams).
hipError_t server_sync(gsc_server* s) {
    hipError_t e = hipStreamSynchronize(s->st);
    if (e == hipSuccess && s->blend_st) e = hipStreamSynchronize(s->blend_st);
    s->blend_pending[0] = s->blend_pending[1] = false;
    return e;
}

// Size the batch raster (both sets with two batches in flight) for the
// admitted viewers (streams must be idle).  The sets only grow while
// viewers remain (a leave keeps them; they go when the last viewer leaves):
// freeing and re-allocating tens of GB stalls the host for up to ~0.6 s,
// which the other viewers' queued frames would wait out.  The budget still
// counts each admitted viewer's share, and the kept size is one the budget
// allowed when it was allocated.
hipError_t resize_raster(gsc_server* s) {
    int64_t e = 0, p = 0, t = 0;
    for (auto& v : s->viewers)
        if (v) {
            e += v->entries;
            p += v->pairs;
            t += v->tiles;
        }
    e = std::min<int64_t>(e, ((int64_t)1 << 31) - 1);
    p = std::min<int64_t>(p, ((int64_t)1 << 31) - 1);
    if (e == s->r_entries && p == s->r_pairs && t == s->r_tiles) return hipSuccess;
    if (e > 0 && e <= s->r_entries && p <= s->r_pairs && t <= s->r_tiles) return hipSuccess;  // fits
    s->rmem.release();
    s->raster = Raster();
    s->rmem2.release();
    s->raster2 = Raster();
    s->r_entries = s->r_pairs = s->r_tiles = 0;
    if (e == 0) return hipSuccess;
    const bool fk = (s->ctx->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0;
    hipError_t err = alloc_raster(s->rmem, s->raster, e, p, t, fk);
    if (err == hipSuccess && s->overlap) err = alloc_raster(s->rmem2, s->raster2, e, p, t, fk);
    if (err != hipSuccess) {
        s->rmem.release();
        s->raster = Raster();
        s->rmem2.release();
        s->raster2 = Raster();
        return err;
    }
    s->r_entries = e;
    s->r_pairs = p;
    s->r_tiles = t;
    return hipSuccess;
}

Viewer* viewer_at(gsc_server* s, int32_t id) {
    if (id < 0 || id >= (int32_t)s->viewers.size()) return nullptr;
    return s->viewers[id].get();
}

}  // namespace

extern "C" {

int gsc_server_create(gsc_ctx* ctx, int64_t budget_bytes, void* stream, gsc_server** out) {
    if (!out) return GSC_E_INVALID_ARG;
    *out = nullptr;
    if (!ctx || budget_bytes <= 0) return GSC_E_INVALID_ARG;
    if (!ctx->loaded) return GSC_E_NOT_LOADED;
    if (ctx->nviews != 1) return GSC_E_INVALID_ARG;  // needs binocular de-redundancy (one view per viewer)
    if ((ctx->cfg.flags & GSC_FLAG_PREDICTOR) && !ctx->pred_loaded) return GSC_E_NOT_LOADED;
    gsc_server* s = new (std::nothrow) gsc_server();
    if (!s) return GSC_E_OOM;
    s->ctx = ctx;
    s->st = (hipStream_t)stream;
    s->budget = budget_bytes;
    *out = s;
    return GSC_OK;
}

void gsc_server_destroy(gsc_server* s) {
    if (!s) return;
    (void)server_sync(s);
    // completion host functions may still be returning on the runtime's thread
    for (int spin = 0; spin < 100000; ++spin) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->in_flight == 0) break;
        }
        timespec ts{0, 100000};
        nanosleep(&ts, nullptr);
    }
    for (auto& v : s->viewers)
        if (v) v->mem.release();
    s->rmem.release();
    s->rmem2.release();
    for (BatchReport* r : s->all_reports) (void)hipHostFree(r);
    for (int i = 0; i < 2; ++i) {
        if (s->front_done[i]) (void)hipEventDestroy(s->front_done[i]);
        if (s->blend_done[i]) (void)hipEventDestroy(s->blend_done[i]);
        if (s->copies_done[i]) (void)hipEventDestroy(s->copies_done[i]);
    }
    if (s->blend_st) (void)hipStreamDestroy(s->blend_st);
    delete s;
}

const char* gsc_server_last_error(const gsc_server* s) { return s ? s->err.c_str() : "null server"; }

int64_t gsc_server_viewer_bytes(gsc_server* s, int32_t max_width, int32_t max_height) {
    if (!s || max_width < 1 || max_height < 1 || max_width > 16384 || max_height > 16384) return GSC_E_INVALID_ARG;
    return (int64_t)viewer_bytes_of(s->ctx, max_width, max_height, s->overlap ? 2 : 1);
}

int gsc_server_admit(gsc_server* s, int32_t max_width, int32_t max_height) {
    if (!s) return GSC_E_INVALID_ARG;
    if (max_width < 1 || max_height < 1 || max_width > 16384 || max_height > 16384)
        return sfail(s, GSC_E_INVALID_ARG, "gsc_server_admit: image size out of range");
    const size_t bytes = viewer_bytes_of(s->ctx, max_width, max_height, s->overlap ? 2 : 1);
    if (s->used + bytes > (size_t)s->budget)
        return sfail(s, GSC_E_BUDGET, "gsc_server_admit: viewer does not fit the device-memory budget now");
    int32_t id = -1;
    for (size_t i = 0; i < s->viewers.size(); ++i)
        if (!s->viewers[i]) {
            id = (int32_t)i;
            break;
        }
    if (id < 0) {
        id = (int32_t)s->viewers.size();
        s->viewers.emplace_back();
    }
    std::unique_ptr<Viewer> v(new (std::nothrow) Viewer());
    if (!v) return sfail(s, GSC_E_OOM, "gsc_server_admit: out of host memory");
    v->max_w = max_width;
    v->max_h = max_height;
    v->bytes = bytes;
    viewer_share(s->ctx, max_width, max_height, v->entries, v->pairs, v->tiles);
    const gsc_ctx* c = s->ctx;
    if (server_sync(s) != hipSuccess) return sfail(s, GSC_E_HIP, "gsc_server_admit: stream failed");
    if (alloc_view(v->mem, v->v, c->scene.n, viewer_cache_lines(c), c->scene.k) != hipSuccess) {
        v->mem.release();
        return sfail(s, GSC_E_OOM, "gsc_server_admit: device allocation");
    }
    if (reset_view(v->v, c->scene.n, c->cfg.d_max, s->st) != hipSuccess) {
        v->mem.release();
        return sfail(s, GSC_E_HIP, "gsc_server_admit: cache reset failed");
    }
    s->viewers[id] = std::move(v);
    {
        std::lock_guard<std::mutex> lk(s->mu);  // completions read it on a runtime thread
        if (s->last_delivered.size() < s->viewers.size()) s->last_delivered.resize(s->viewers.size());
        s->last_delivered[(size_t)id] = -INFINITY;
    }
    if (resize_raster(s) != hipSuccess) {
        s->viewers[id]->mem.release();
        s->viewers[id].reset();
        (void)resize_raster(s);
        return sfail(s, GSC_E_OOM, "gsc_server_admit: raster allocation");
    }
    s->used += bytes;
    return id;
}

int64_t gsc_server_submit(gsc_server* s, int32_t viewer, const gsc_camera* left, const gsc_camera* right,
                          double t_arrival, float* out_left, float* out_right) {
    if (!s) return GSC_E_INVALID_ARG;
    Viewer* v = viewer_at(s, viewer);
    if (!v) return sfail(s, GSC_E_INVALID_ARG, "gsc_server_submit: no such viewer");
    if (!left || !right || !out_left || !out_right) return sfail(s, GSC_E_INVALID_ARG, "gsc_server_submit: null argument");
    if (!valid_camera(*left) || !valid_camera(*right))
        return sfail(s, GSC_E_INVALID_ARG, "gsc_server_submit: invalid camera");
    if (left->width != right->width || left->height != right->height || left->fovx != right->fovx ||
        left->fovy != right->fovy || left->znear != right->znear)
        return sfail(s, GSC_E_INVALID_ARG, "gsc_server_submit: eyes must share intrinsics");
    if (left->width > v->max_w || left->height > v->max_h)
        return sfail(s, GSC_E_INVALID_ARG, "gsc_server_submit: image larger than the viewer's admitted size");
    Request r;
    r.eye[0] = *left;
    r.eye[1] = *right;
    unified_camera(*left, *right, r.unified);
    // viewing direction: the camera's z axis in world coordinates (third row
    // of the world-to-camera rotation)
    const double dir[3] = {r.unified.R[6], r.unified.R[7], r.unified.R[8]};
    if ((s->pose_m > 0.0 || s->pose_rad > 0.0) && v->has_pose) {
        double d2 = 0.0, dot = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double dp = r.unified.pos[k] - v->pose[k];
            d2 += dp * dp;
            dot += dir[k] * v->dir[k];
        }
        const double ang = std::acos(std::max(-1.0, std::min(1.0, dot)));
        const bool moved = s->pose_m > 0.0 && std::sqrt(d2) > s->pose_m;
        const bool turned = s->pose_rad > 0.0 && ang > s->pose_rad;
        if (!moved && !turned) return sfail(s, GSC_E_UNCHANGED, "gsc_server_submit: pose change below the threshold");
    }
    v->has_pose = true;
    for (int k = 0; k < 3; ++k) {
        v->pose[k] = r.unified.pos[k];
        v->dir[k] = dir[k];
    }
    r.id = s->next_id++;
    r.t_arrival = t_arrival;
    r.out[0] = out_left;
    r.out[1] = out_right;
    v->queue.push_back(r);
    return r.id;
}

int gsc_server_step(gsc_server* s) {
    if (!s) return GSC_E_INVALID_ARG;
    gsc_ctx* c = s->ctx;
    // queue timeout: requests waited too long are dropped unrendered
    if (s->timeout_s > 0.0) {
        const double now = now_monotonic();
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& vp : s->viewers) {
            if (!vp) continue;
            while (!vp->queue.empty() && now - vp->queue.front().t_arrival > s->timeout_s) {
                s->done.push_back({vp->queue.front().id, now, GSC_E_TIMEOUT});
                vp->queue.pop_front();
            }
        }
    }
    // oldest head request first, one request per viewer per batch
    std::vector<int32_t> pick;
    for (int32_t i = 0; i < (int32_t)s->viewers.size(); ++i)
        if (s->viewers[i] && !s->viewers[i]->queue.empty()) pick.push_back(i);
    if (pick.empty()) return 0;
    std::stable_sort(pick.begin(), pick.end(), [&](int32_t a, int32_t b) {
        return s->viewers[a]->queue.front().t_arrival < s->viewers[b]->queue.front().t_arrival;
    });
    if ((int)pick.size() > kMaxBatchViewers) pick.resize(kMaxBatchViewers);

    BatchReport* rep = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->free_reports.empty()) {
            rep = s->free_reports.back();
            s->free_reports.pop_back();
        }
    }
    if (!rep) {
        if (hipHostMalloc((void**)&rep, sizeof(BatchReport)) != hipSuccess)
            return sfail(s, GSC_E_OOM, "gsc_server_step: pinned allocation");
        s->all_reports.push_back(rep);
    }
    Batch* b = new (std::nothrow) Batch();
    if (!b) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->free_reports.push_back(rep);
        return sfail(s, GSC_E_OOM, "gsc_server_step: out of host memory");
    }
    b->s = s;
    b->rep = rep;
    b->nviewers = (int)pick.size();

    SegTable tab;
    std::memset(&tab, 0, sizeof(tab));
    tab.paired = 1;  // each viewer's two eyes read its one view
    int tiles = 0;
    for (int i = 0; i < (int)pick.size(); ++i) {
        Viewer& v = *s->viewers[pick[i]];
        Request r = v.queue.front();
        v.queue.pop_front();
        DeriveArgs a;
        a.sc = &c->scene;
        a.v = &v.v;
        a.cam = derive_cam(r.unified, c->scene.d_ref, (c->cfg.flags & GSC_FLAG_LOD_FADE) != 0);
        a.precision = c->cfg.precision;
        a.flags = c->cfg.flags;
        a.d_max = c->cfg.d_max;
        a.guide = c->cfg.guide;
        a.pred_thr = c->cfg.predictor_threshold;
        a.pred_w = c->pred_w;
        a.pred_wbf = c->pred_wbf;
        a.collect = 0;
        b->ids.push_back(r.id);
        b->viewer_of.push_back(i);
        b->viewer_id.push_back(pick[i]);
        b->t_arrival.push_back(r.t_arrival);
        hipError_t e = derive_frame(a, s->st);
        if (e != hipSuccess)
            return abort_batch(s, b, std::string("gsc_server_step: derive: ") + hipGetErrorString(e));
        v.v.t += 1;
        for (int eye = 0; eye < 2; ++eye) {
            Seg& sg = tab.s[tab.n++];
            sg.L0 = v.v.L0; sg.L1 = v.v.L1; sg.L2 = v.v.L2; sg.L3 = v.v.L3;
            const bool direct = (c->cfg.flags & GSC_FLAG_REUSE) && v.v.C >= c->scene.n;  // line a = anchor a
            sg.anchor_pos = c->scene.posr; sg.line_anchor = direct ? nullptr : v.v.line_anchor; sg.k = c->scene.k;
            sg.G = v.v.G; sg.nG = &v.v.cnt->n_gauss; sg.nG_host = 0;
            seg_camera(sg, r.eye[eye]);
            if (c->cfg.flags & GSC_FLAG_LOD_FADE) seg_lod_fade(sg, c->scene, r.unified);
            sg.tile_base = tiles;
            tiles += sg.ntx * sg.nty;
            sg.out_rgb = r.out[eye];
            sg.out_T = nullptr;
            sg.out_nc = nullptr;
        }
        if (hipMemcpyAsync(&rep->vc[i], v.v.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s->st) != hipSuccess)
            return abort_batch(s, b, "gsc_server_step: counter copy");
    }
    tab.total_tiles = tiles;
    // two batches in flight: this batch's raster set was last read by the
    // blend two batches back, which must finish before the preprocess
    // rewrites it; this batch's blend then runs on the blend stream
    const int set = s->overlap ? (int)(s->nbatch & 1) : 0;
    Raster& R = set ? s->raster2 : s->raster;
    hipError_t e = hipSuccess;
    if (s->overlap && s->blend_pending[set]) e = hipStreamWaitEvent(s->st, s->blend_done[set], 0);
    if (e == hipSuccess)
        e = raster_batch(tab, R, (c->cfg.flags & GSC_FLAG_FULL_KEY_SORT) != 0, false, s->st, nullptr,
                         s->overlap ? s->blend_st : nullptr, s->overlap ? s->front_done[set] : nullptr);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&rep->rc, R.cnt, sizeof(RasterCounters), hipMemcpyDeviceToHost, s->st);
    hipStream_t done_st = s->st;
    if (e == hipSuccess && s->overlap) {
        // completion after the blend and after the counter copies on the
        // server's stream
        e = hipEventRecord(s->blend_done[set], s->blend_st);
        if (e == hipSuccess) s->blend_pending[set] = true;
        if (e == hipSuccess) e = hipEventRecord(s->copies_done[set], s->st);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->blend_st, s->copies_done[set], 0);
        done_st = s->blend_st;
    }
    if (e != hipSuccess) return abort_batch(s, b, std::string("gsc_server_step: raster: ") + hipGetErrorString(e));
    s->nbatch += 1;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->in_flight += 1;
    }
    const int launched = (int)b->ids.size();
    e = hipLaunchHostFunc(done_st, on_batch_done, b);
    if (e != hipSuccess) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->in_flight -= 1;
        }
        return abort_batch(s, b, "gsc_server_step: completion callback");
    }
    return launched;
}

int gsc_server_poll(gsc_server* s, int64_t* ids, double* t_done, int32_t* status, int32_t cap) {
    if (!s || cap < 0 || (cap > 0 && (!ids || !t_done))) return GSC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    const int32_t m = (int32_t)std::min<size_t>((size_t)cap, s->done.size());
    for (int32_t i = 0; i < m; ++i) {
        ids[i] = s->done[i].id;
        t_done[i] = s->done[i].t;
        if (status) status[i] = s->done[i].status;
    }
    s->done.erase(s->done.begin(), s->done.begin() + m);
    return m;
}

int gsc_server_policy(gsc_server* s, double pose_m, double pose_rad, double timeout_s, int ordered) {
    if (!s) return GSC_E_INVALID_ARG;
    if (!std::isfinite(pose_m) || !std::isfinite(pose_rad) || !std::isfinite(timeout_s))
        return sfail(s, GSC_E_INVALID_ARG, "gsc_server_policy: non-finite argument");
    std::lock_guard<std::mutex> lk(s->mu);
    s->pose_m = pose_m;
    s->pose_rad = pose_rad;
    s->timeout_s = timeout_s;
    s->ordered = ordered != 0;
    return GSC_OK;
}

int gsc_server_overlap(gsc_server* s, int enable) {
    if (!s) return GSC_E_INVALID_ARG;
    for (auto& v : s->viewers)
        if (v) return sfail(s, GSC_E_INVALID_ARG, "gsc_server_overlap: set before admitting viewers");
    if (server_sync(s) != hipSuccess) return sfail(s, GSC_E_HIP, "gsc_server_overlap: stream failed");
    if (enable && !s->blend_st) {
        if (hipStreamCreateWithFlags(&s->blend_st, hipStreamNonBlocking) != hipSuccess)
            return sfail(s, GSC_E_HIP, "gsc_server_overlap: stream creation");
        for (int i = 0; i < 2; ++i)
            if (hipEventCreateWithFlags(&s->front_done[i], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s->blend_done[i], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s->copies_done[i], hipEventDisableTiming) != hipSuccess)
                return sfail(s, GSC_E_HIP, "gsc_server_overlap: event creation");
    }
    s->overlap = enable != 0;
    s->nbatch = 0;
    return GSC_OK;
}

int gsc_server_pending(gsc_server* s) {
    if (!s) return GSC_E_INVALID_ARG;
    int64_t q = 0;
    for (auto& v : s->viewers)
        if (v) q += (int64_t)v->queue.size();
    std::lock_guard<std::mutex> lk(s->mu);
    return (int)std::min<int64_t>(q + s->in_flight, 1 << 30);
}

int gsc_server_leave(gsc_server* s, int32_t viewer) {
    if (!s) return GSC_E_INVALID_ARG;
    Viewer* v = viewer_at(s, viewer);
    if (!v) return sfail(s, GSC_E_INVALID_ARG, "gsc_server_leave: no such viewer");
    if (!v->queue.empty()) return sfail(s, GSC_E_INVALID_ARG, "gsc_server_leave: viewer has queued requests");
    if (server_sync(s) != hipSuccess) return sfail(s, GSC_E_HIP, "gsc_server_leave: stream failed");
    s->used -= v->bytes;
    v->mem.release();
    s->viewers[viewer].reset();
    if (resize_raster(s) != hipSuccess) return sfail(s, GSC_E_OOM, "gsc_server_leave: raster allocation");
    return GSC_OK;
}

}  // extern "C"
