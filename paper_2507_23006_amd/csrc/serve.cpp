// Level-of-detail selection and the serving runtime (declared in gs.h).
//
// Selection is host code over the partition table (§3.4.2: levels are
// chosen per render-time partition from the partition-camera distance,
// invisible partitions are culled; Tab. 13: the thresholds are the largest
// distances at which each level is used).  The budget rule is this
// library's own: the paper caps Gaussians per partition while training, a
// served request caps the total it renders.
//
// The server is a FIFO of requests and a pool of worker threads, each with
// its own HIP stream and device buffers.  A free worker takes every arrived
// request at the head of the queue that fits its capacities (continuous
// batching), projects each view's selected level segments with one
// segment-table launch, sorts all views' pairs together and composites them
// in one multi-view launch.  Views never share tiles, and each view's slots
// keep the order of its own segment list, so an image does not depend on
// the batch it was rendered in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "gs.h"
#include "gs_internal.h"
#include "host.h"

using namespace gs;
using namespace gs::host;

namespace {

struct Lod {
    int L = 0, P = 0;
    std::vector<float> pmin, pmax;
    std::vector<int64_t> off, cnt;
    double th[GS_MAX_LEVELS];
    double margin = 0.0;
};

int copy_table(const gs_lod_table* t, Lod* out) {
    GS_REQUIRE(t != nullptr, "lod table is NULL");
    GS_REQUIRE(t->n_levels >= 1 && t->n_levels <= GS_MAX_LEVELS, "n_levels=%d outside 1..%d", t->n_levels,
               GS_MAX_LEVELS);
    GS_REQUIRE(t->n_parts >= 1, "n_parts=%d must be >= 1", t->n_parts);
    GS_REQUIRE(t->part_min && t->part_max && t->offsets && t->counts, "lod table array is NULL");
    GS_REQUIRE(std::isfinite(t->margin) && t->margin >= 0.0f, "margin must be finite and >= 0");
    const int L = t->n_levels, P = t->n_parts;
    for (int k = 0; k < L; ++k) {
        GS_REQUIRE(!std::isnan(t->thresholds[k]) && t->thresholds[k] >= 0.0f, "threshold %d is not >= 0", k);
        GS_REQUIRE(k == 0 || t->thresholds[k] >= t->thresholds[k - 1], "thresholds must not decrease");
    }
    for (int64_t i = 0; i < (int64_t)L * P; ++i)
        GS_REQUIRE(t->offsets[i] >= 0 && t->counts[i] >= 0, "negative offset or count at %lld", (long long)i);
    for (int64_t i = 0; i < 3LL * P; ++i)
        GS_REQUIRE(std::isfinite(t->part_min[i]) && std::isfinite(t->part_max[i]) && t->part_min[i] <= t->part_max[i],
                   "partition box %lld malformed", (long long)(i / 3));
    out->L = L;
    out->P = P;
    out->pmin.assign(t->part_min, t->part_min + 3 * P);
    out->pmax.assign(t->part_max, t->part_max + 3 * P);
    out->off.assign(t->offsets, t->offsets + (size_t)L * P);
    out->cnt.assign(t->counts, t->counts + (size_t)L * P);
    for (int k = 0; k < GS_MAX_LEVELS; ++k) out->th[k] = k < L ? (double)t->thresholds[k] : INFINITY;
    out->margin = t->margin;
    return GS_OK;
}

int check_camera(const gs_camera* c) {
    ViewTable vt;
    return build_views(c, 1, &vt);
}

// frustum of a camera as five half-spaces f(p) >= 0 in camera coordinates
struct Frustum {
    double R[9], t[3], c[3];
    double ulo, uhi, vlo, vhi, znear;
};

Frustum frustum_of(const gs_camera& cam) {
    Frustum f;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) f.R[3 * r + k] = cam.viewmat[4 * r + k];
        f.t[r] = cam.viewmat[4 * r + 3];
    }
    for (int i = 0; i < 3; ++i) f.c[i] = -(f.R[i] * f.t[0] + f.R[3 + i] * f.t[1] + f.R[6 + i] * f.t[2]);
    const double W = cam.width, H = cam.height;
    f.ulo = -(cam.cx + 0.15 * W) / cam.fx;
    f.uhi = (W - cam.cx + 0.15 * W) / cam.fx;
    f.vlo = -(cam.cy + 0.15 * H) / cam.fy;
    f.vhi = (H - cam.cy + 0.15 * H) / cam.fy;
    f.znear = cam.near_plane;
    return f;
}

// false when the box [lo - m, hi + m] lies entirely on the outer side of one plane
bool box_in_view(const Frustum& f, const float* lo, const float* hi, double m) {
    bool out_plane[5] = {true, true, true, true, true};
    for (int i = 0; i < 8; ++i) {
        const double x[3] = {(i & 1) ? hi[0] + m : lo[0] - m, (i & 2) ? hi[1] + m : lo[1] - m,
                             (i & 4) ? hi[2] + m : lo[2] - m};
        double p[3];
        for (int r = 0; r < 3; ++r) p[r] = f.R[3 * r] * x[0] + f.R[3 * r + 1] * x[1] + f.R[3 * r + 2] * x[2] + f.t[r];
        const double g[5] = {p[2] - f.znear, p[0] - f.ulo * p[2], f.uhi * p[2] - p[0], p[1] - f.vlo * p[2],
                             f.vhi * p[2] - p[1]};
        for (int k = 0; k < 5; ++k) out_plane[k] = out_plane[k] && g[k] < 0.0;
    }
    for (int k = 0; k < 5; ++k)
        if (out_plane[k]) return false;
    return true;
}

double box_distance(const double c[3], const float* lo, const float* hi) {
    double d2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double e = std::max({(double)lo[i] - c[i], 0.0, c[i] - (double)hi[i]});
        d2 += e * e;
    }
    return std::sqrt(d2);
}

int lod_select(const Lod& t, const gs_camera& cam, int64_t budget, int32_t* level, int64_t* total_out) {
    const int L = t.L, P = t.P;
    const Frustum f = frustum_of(cam);
    std::vector<double> dist(P, 0.0);
    int64_t total = 0;
    auto count = [&](int p, int l) { return l > 0 ? t.cnt[(size_t)(l - 1) * P + p] : (int64_t)0; };
    bool any_visible = false;
    for (int p = 0; p < P; ++p) {
        level[p] = 0;
        if (!box_in_view(f, &t.pmin[3 * p], &t.pmax[3 * p], t.margin)) continue;
        any_visible = true;
        dist[p] = box_distance(f.c, &t.pmin[3 * p], &t.pmax[3 * p]);
        int l = 1;
        for (int k = 0; k < L; ++k)
            if (dist[p] <= t.th[k]) {
                l = L - k;
                break;
            }
        level[p] = l;
        total += count(p, l);
    }
    if (total > budget) {
        // farthest first, ties by lower id
        std::vector<int> order(P);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dist[a] > dist[b]; });
        // each pass takes the partitions at the finest level in use down one
        // level, farthest first, until the total fits
        for (int top = L; top >= 2 && total > budget; --top)
            for (int i = 0; i < P && total > budget; ++i) {
                const int p = order[i];
                if (level[p] != top) continue;
                total += count(p, top - 1) - count(p, top);
                level[p] = top - 1;
            }
        for (int i = 0; i < P && total > budget; ++i) {
            const int p = order[i];
            if (level[p] == 0) continue;
            total -= count(p, level[p]);
            level[p] = 0;
        }
        bool kept = false;
        for (int p = 0; p < P; ++p) kept = kept || level[p] > 0;
        if (any_visible && !kept)
            return fail(GS_ERR_BUDGET, "budget %lld cannot hold the nearest visible partition", (long long)budget);
    }
    *total_out = total;
    return GS_OK;
}

double tiles_of(const gs_camera& c) {
    return (double)((c.width + kTile - 1) / kTile) * (double)((c.height + kTile - 1) / kTile);
}

}  // namespace

struct Request {
    uint64_t ticket;
    gs_camera cam;
    int64_t budget;
    float* out;
    hipEvent_t ready = nullptr;   // recorded on the caller's stream at submit
    double t_arrival;
    std::vector<int32_t> level;
    int64_t n_sel, n_pix, n_tiles;
};

// One set of a worker's device buffers and the batch it holds in flight.
struct BufSet {
    Projected proj{};
    SlotSeg* segs_dev = nullptr;
    SlotSeg* segs_host = nullptr;
    uint32_t* pairs = nullptr;
    uint32_t* ranges = nullptr;
    void* bin_ws = nullptr;
    size_t bin_ws_bytes = 0;
    float *rgb = nullptr, *depth = nullptr, *alpha = nullptr, *T = nullptr;
    int32_t* last = nullptr;
    int64_t* npairs_dev = nullptr;      // the binning's pair count (device)
    int64_t* npairs_host = nullptr;     // its copy after the batch (pinned)
    uint32_t* work = nullptr;           // work counter of persistent compositing
    void* seg = nullptr;                // segment area of the segmented forward
    size_t seg_bytes = 0;
    hipEvent_t prepped = nullptr;       // projection and binning done
    hipEvent_t done = nullptr;          // images and pair count written
    // the batch in flight
    std::vector<Request> reqs;
    int64_t slots = 0;
    int64_t pair_bound = 0;             // the binning's pair bound for this batch
    double est_pairs = 0.0, t_start = 0.0;
    int rc = GS_OK;
};

struct Worker {
    gs_server* srv = nullptr;
    hipStream_t prep = nullptr;         // projection and binning
    hipStream_t render = nullptr;       // compositing and output copies
    std::vector<BufSet> sets;
    std::thread th;
};

struct gs_server {
    GaussPtrs gp{};
    int64_t n = 0;
    Lod lod;
    OptK opt{};
    gs_serve_config cfg{};
    int64_t tile_cap = 0, seg_cap = 0;
    int device = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t submitted = 0;
    // admission model (under mu): pairs per selected Gaussian by resolution
    std::map<uint64_t, double> ratio;
    std::vector<hipEvent_t> free_events;

    std::mutex done_mu;
    std::condition_variable done_cv;
    std::deque<gs_completion> done;
    std::vector<double> lat_ms;
    int64_t completed = 0, failed = 0, batches = 0, batch_views = 0, pixels = 0, split_batches = 0,
            rebinned_batches = 0;
    double first_arrival = INFINITY, last_done = 0.0, est_over_actual = 0.0;
    int64_t est_batches = 0;

    std::vector<Worker*> workers;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

// headroom of the admission estimate over the learned ratio
constexpr double kAdmitMargin = 1.15;
// a batch bins with a pair bound of its estimate times kBoundMargin plus
// kBoundFloor (at most the pair capacity): the binning launches are sized
// by that bound, so a lone small request does not pay for grids sized for
// the whole pair buffer; a count above it re-bins at the full capacity
constexpr double kBoundMargin = 1.5;
constexpr int64_t kBoundFloor = 4096;
constexpr double kDefaultPairsPerGaussian = 8.0;

uint64_t view_class(const gs_camera& c) { return ((uint64_t)(uint32_t)c.width << 32) | (uint32_t)c.height; }

// estimated pairs of one request (caller holds s->mu)
double estimate_pairs(const gs_server* s, const Request& r) {
    const auto it = s->ratio.find(view_class(r.cam));
    double k = s->cfg.pairs_per_gaussian > 0.0 ? s->cfg.pairs_per_gaussian : kDefaultPairsPerGaussian;
    if (it != s->ratio.end()) k = it->second;
    return (double)r.n_sel * k;
}

// after a batch: scale the ratios of its view classes by observed/estimated,
// at once upward, a quarter of the way downward
void learn_pairs(gs_server* s, const Request* r, int nb, int64_t observed) {
    std::lock_guard<std::mutex> lk(s->mu);
    double est = 0.0;
    for (int i = 0; i < nb; ++i) est += estimate_pairs(s, r[i]);
    if (est <= 0.0) return;
    const double f = (double)observed / est;
    const double g = f >= 1.0 ? f : 1.0 - 0.25 * (1.0 - f);
    std::vector<uint64_t> seen;
    for (int i = 0; i < nb; ++i) {
        const uint64_t c = view_class(r[i].cam);
        if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
        seen.push_back(c);
        const auto it = s->ratio.find(c);
        const double k = it != s->ratio.end() ? it->second
                         : (s->cfg.pairs_per_gaussian > 0.0 ? s->cfg.pairs_per_gaussian : kDefaultPairsPerGaussian);
        s->ratio[c] = std::max(k * g, 1e-3);
    }
}

void recycle_events(gs_server* s, Request* r, int nb) {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int i = 0; i < nb; ++i)
        if (r[i].ready) {
            s->free_events.push_back(r[i].ready);
            r[i].ready = nullptr;
        }
}

void free_set(BufSet& b) {
    void* dev[] = {b.proj.rec, b.proj.rect, b.proj.tiles, b.proj.dkey, b.proj.tile_order, b.proj.tile_mask,
                   b.segs_dev, b.pairs,     b.ranges,     b.bin_ws,    b.rgb,              b.depth,
                   b.alpha,    b.T,         b.last,       b.npairs_dev, b.work,           b.seg};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (b.segs_host) (void)hipHostFree(b.segs_host);
    if (b.npairs_host) (void)hipHostFree(b.npairs_host);
    if (b.prepped) (void)hipEventDestroy(b.prepped);
    if (b.done) (void)hipEventDestroy(b.done);
}

void free_worker(Worker* w) {
    if (!w) return;
    for (BufSet& b : w->sets) free_set(b);
    if (w->prep) (void)hipStreamDestroy(w->prep);
    if (w->render) (void)hipStreamDestroy(w->render);
    delete w;
}

template <class T>
hipError_t dev_alloc(T** p, size_t count) {
    return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

int alloc_set(gs_server* s, BufSet& b) {
    const int64_t S = s->cfg.slot_capacity, Pc = s->cfg.pair_capacity, X = s->cfg.pixel_capacity;
    GS_HIP(dev_alloc(&b.proj.rec, 4 * (size_t)S));
    GS_HIP(dev_alloc(&b.proj.rect, (size_t)S));
    GS_HIP(dev_alloc(&b.proj.tiles, (size_t)S));
    GS_HIP(dev_alloc(&b.proj.dkey, (size_t)S));
    GS_HIP(dev_alloc(&b.proj.tile_mask, (size_t)S));
    GS_HIP(dev_alloc(&b.segs_dev, (size_t)s->seg_cap));
    GS_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.segs_host), (size_t)s->seg_cap * sizeof(SlotSeg),
                         hipHostMallocDefault));
    GS_HIP(dev_alloc(&b.pairs, (size_t)Pc));
    GS_HIP(dev_alloc(&b.ranges, 2 * (size_t)s->tile_cap));
    GS_HIP(dev_alloc(&b.proj.tile_order, (size_t)s->tile_cap));
    b.bin_ws_bytes = bin_workspace_bytes(S, Pc);
    GS_HIP(hipMalloc(&b.bin_ws, b.bin_ws_bytes));
    GS_HIP(dev_alloc(&b.rgb, 3 * (size_t)X));
    GS_HIP(dev_alloc(&b.depth, (size_t)X));
    GS_HIP(dev_alloc(&b.alpha, (size_t)X));
    GS_HIP(dev_alloc(&b.T, (size_t)X));
    GS_HIP(dev_alloc(&b.last, (size_t)X));
    GS_HIP(dev_alloc(&b.npairs_dev, 1));
    GS_HIP(dev_alloc(&b.work, 1));
    b.seg_bytes = gs_seg_workspace_size(s->tile_cap, Pc);
    GS_HIP(hipMalloc(&b.seg, b.seg_bytes));
    GS_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.npairs_host), sizeof(int64_t), hipHostMallocDefault));
    GS_HIP(hipEventCreateWithFlags(&b.prepped, hipEventDisableTiming));
    GS_HIP(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    return GS_OK;
}

int alloc_worker(gs_server* s, Worker* w) {
    GS_HIP(hipStreamCreateWithFlags(&w->prep, hipStreamNonBlocking));
    GS_HIP(hipStreamCreateWithFlags(&w->render, hipStreamNonBlocking));
    w->sets.resize((size_t)s->cfg.pipeline_depth);
    for (BufSet& b : w->sets) {
        const int rc = alloc_set(s, b);
        if (rc) return rc;
    }
    return GS_OK;
}

// Enqueues views r[0..nb) as one batch into buffer set b: projection and
// binning on the prep stream, compositing and the copies into the callers'
// images on the render stream (after each request's ready event).  Returns
// without waiting; b.done marks the end of the batch's work.
int launch_batch(Worker* w, BufSet& b, Request* r, int nb, bool full_bound = false) {
    gs_server* s = w->srv;
    gs_camera cams[GS_MAX_VIEWS];
    for (int i = 0; i < nb; ++i) cams[i] = r[i].cam;
    ViewTable vt;
    int rc = build_views(cams, nb, &vt);
    if (rc) return rc;
    const int P = s->lod.P;
    int ns = 0;
    int64_t slots = 0;
    for (int v = 0; v < nb; ++v)
        for (int p = 0; p < P; ++p) {
            const int l = r[v].level[p];
            if (l <= 0) continue;
            const size_t k = (size_t)(l - 1) * P + p;
            const int64_t c = s->lod.cnt[k];
            if (c == 0) continue;
            b.segs_host[ns++] = SlotSeg{s->lod.off[k], (uint32_t)slots, (uint32_t)v};
            slots += c;
        }
    if (slots > s->cfg.slot_capacity) return fail(GS_ERR_CAPACITY, "batch selects %lld Gaussians", (long long)slots);
    b.slots = slots;
    b.pair_bound = s->cfg.pair_capacity;
    if (!full_bound) {
        double est = 0.0;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (int i = 0; i < nb; ++i) est += estimate_pairs(s, r[i]);
        }
        const double bound = est * kBoundMargin + (double)kBoundFloor;
        if (bound < (double)b.pair_bound) b.pair_bound = (int64_t)bound;
    }
    if (slots > 0) {
        GS_HIP(hipMemcpyAsync(b.segs_dev, b.segs_host, (size_t)ns * sizeof(SlotSeg), hipMemcpyHostToDevice, w->prep));
        GS_HIP(launch_project_slots(s->gp, s->n, vt, s->opt, b.segs_dev, ns, (uint32_t)slots, b.proj, w->prep));
        rc = bin_sort_slots(b.proj, vt, slots, b.pair_bound, b.pairs, b.ranges, b.npairs_dev, b.bin_ws,
                            b.bin_ws_bytes, w->prep);
        if (rc) return rc;
        GS_HIP(hipEventRecord(b.prepped, w->prep));
        GS_HIP(hipStreamWaitEvent(w->render, b.prepped, 0));
    } else {
        GS_HIP(fill_u32(b.ranges, 0u, 2 * (size_t)vt.total_tiles, w->render));
        GS_HIP(launch_tile_order(b.ranges, (uint32_t)vt.total_tiles, b.proj.tile_order, w->render));
    }
    // long lists composited in segments (one workgroup per tile when the
    // compositing is persistent)
    SegPlan plan;
    uint32_t cap = 0;
    seg_layout(b.seg, b.seg_bytes, vt.total_tiles, &plan, &cap);
    const bool segmented = plan.work_off && slots > 0 && s->cfg.persistent_ctas == 0;
    if (segmented)
        GS_HIP(launch_seg_plan(b.proj, reinterpret_cast<const uint2*>(b.ranges), vt, cap, plan, w->render));
    GS_HIP(launch_render_fwd(b.proj, b.pairs, reinterpret_cast<const uint2*>(b.ranges), vt, s->opt, b.rgb, b.depth,
                             b.alpha, b.T, b.last, w->render, s->cfg.persistent_ctas, b.work,
                             segmented ? &plan : nullptr));
    for (int v = 0; v < nb; ++v) {
        if (r[v].ready) GS_HIP(hipStreamWaitEvent(w->render, r[v].ready, 0));
        GS_HIP(hipMemcpyAsync(r[v].out, b.rgb + 3 * vt.v[v].pix_off,
                              (size_t)r[v].cam.width * r[v].cam.height * 3 * sizeof(float), hipMemcpyDeviceToDevice,
                              w->render));
    }
    if (slots > 0)
        GS_HIP(hipMemcpyAsync(b.npairs_host, b.npairs_dev, sizeof(int64_t), hipMemcpyDeviceToHost, w->render));
    GS_HIP(hipEventRecord(b.done, w->render));
    return GS_OK;
}

// Waits for the batch in b; *n_pairs gets its pair count.  GS_ERR_CAPACITY
// when the pairs overflowed the batch's bound (the lists were left empty).
int wait_batch(Worker* w, BufSet& b, int launch_rc, int64_t* n_pairs) {
    gs_server* s = w->srv;
    *n_pairs = 0;
    if (launch_rc) {
        // drain whatever part of the batch was enqueued
        (void)hipStreamSynchronize(w->prep);
        (void)hipStreamSynchronize(w->render);
        return launch_rc;
    }
    GS_HIP(hipEventSynchronize(b.done));
    if (b.slots > 0) {
        *n_pairs = *b.npairs_host;
        if (*n_pairs > b.pair_bound)
            return fail(GS_ERR_CAPACITY, "batch needs %lld pairs (bound %lld, capacity %lld)", (long long)*n_pairs,
                        (long long)b.pair_bound, (long long)s->cfg.pair_capacity);
    }
    return GS_OK;
}

void complete(gs_server* s, Request* r, int nb, int status, int64_t n_pairs, double t_start, double t_done) {
    recycle_events(s, r, nb);
    std::lock_guard<std::mutex> lk(s->done_mu);
    s->batches += 1;
    s->batch_views += nb;
    for (int i = 0; i < nb; ++i) {
        gs_completion c{};
        c.ticket = r[i].ticket;
        c.status = status;
        c.batch_views = nb;
        c.n_gaussians = r[i].n_sel;
        c.n_pairs = n_pairs;
        c.t_arrival = r[i].t_arrival;
        c.t_start = t_start;
        c.t_done = t_done;
        s->done.push_back(c);
        if (status == GS_OK) {
            s->completed += 1;
            s->pixels += r[i].n_pix;
            s->lat_ms.push_back((t_done - r[i].t_arrival) * 1e3);
            s->first_arrival = std::min(s->first_arrival, r[i].t_arrival);
            s->last_done = std::max(s->last_done, t_done);
        } else {
            s->failed += 1;
        }
    }
    s->done_cv.notify_all();
}

void note_estimate(gs_server* s, double est, int64_t observed) {
    if (observed <= 0) return;
    std::lock_guard<std::mutex> lk(s->done_mu);
    s->est_over_actual += est / (double)observed;
    s->est_batches += 1;
}

// Settles a batch whose launch returned launch_rc: waits for it, learns its
// pair ratio, and completes its requests -- or, when it overflowed a buffer,
// renders its halves one after the other in the same buffer set.
void settle(Worker* w, BufSet& b, Request* r, int nb, int launch_rc, double t_start, double est) {
    gs_server* s = w->srv;
    int64_t n_pairs = 0;
    int rc;
    try {
        rc = wait_batch(w, b, launch_rc, &n_pairs);
    } catch (...) {
        rc = GS_ERR_INTERNAL;
    }
    if (n_pairs > 0) {
        if (est > 0.0) note_estimate(s, est, n_pairs);
        learn_pairs(s, r, nb, n_pairs);
    }
    if (rc == GS_ERR_CAPACITY && n_pairs > 0 && n_pairs <= s->cfg.pair_capacity && b.pair_bound < s->cfg.pair_capacity) {
        // the estimate fell short of the count: bin again with the whole buffer
        {
            std::lock_guard<std::mutex> lk(s->done_mu);
            s->rebinned_batches += 1;
        }
        int lrc;
        try {
            lrc = launch_batch(w, b, r, nb, /*full_bound=*/true);
        } catch (...) {
            lrc = GS_ERR_INTERNAL;
        }
        settle(w, b, r, nb, lrc, t_start, -1.0);
        return;
    }
    if (rc == GS_ERR_CAPACITY && nb > 1) {
        {
            std::lock_guard<std::mutex> lk(s->done_mu);
            s->split_batches += 1;
        }
        const int h = nb / 2;
        for (int part = 0; part < 2; ++part) {
            Request* q = part ? r + h : r;
            const int m = part ? nb - h : h;
            const double t = s->now();
            int lrc;
            try {
                lrc = launch_batch(w, b, q, m);
            } catch (...) {
                lrc = GS_ERR_INTERNAL;
            }
            settle(w, b, q, m, lrc, t, -1.0);
        }
        return;
    }
    complete(s, r, nb, rc, n_pairs, t_start, s->now());
}

// Takes every arrived request at the head of the queue that fits one batch:
// views, slots, pixels, tiles, and the estimated pairs against the pair
// buffer (the first request always).  With `block`, waits for an arrival.
// Returns false once the server stops.
bool take_batch(gs_server* s, bool block, std::vector<Request>* batch, double* est_out) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stop) return false;
        if (!s->queue.empty()) {
            const double wait = s->queue.front().t_arrival - s->now();
            if (wait <= 0.0) break;
            if (!block) return true;
            s->cv.wait_for(lk, std::chrono::duration<double>(wait));
        } else {
            if (!block) return true;
            s->cv.wait(lk);
        }
    }
    int64_t slots = 0, pix = 0, tiles = 0;
    double est = 0.0;
    const double now = s->now(), pair_room = (double)s->cfg.pair_capacity;
    while (!s->queue.empty() && (int)batch->size() < s->cfg.max_views_per_batch) {
        Request& q = s->queue.front();
        if (q.t_arrival > now) break;
        const double e = estimate_pairs(s, q);
        if (!batch->empty() &&
            (slots + q.n_sel > s->cfg.slot_capacity || pix + q.n_pix > s->cfg.pixel_capacity ||
             tiles + q.n_tiles > s->tile_cap || (est + e) * kAdmitMargin > pair_room))
            break;
        slots += q.n_sel;
        pix += q.n_pix;
        tiles += q.n_tiles;
        est += e;
        batch->push_back(std::move(q));
        s->queue.pop_front();
    }
    *est_out = est;
    lk.unlock();
    s->cv.notify_all();
    return true;
}

// A worker keeps up to pipeline_depth batches in flight, one per buffer
// set: while batch k composites on the render stream, batch k+1 projects and
// bins on the prep stream.  Batches are settled in launch order.
void worker_main(Worker* w) {
    gs_server* s = w->srv;
    (void)hipSetDevice(s->device);
    const int D = (int)w->sets.size();
    std::deque<int> inflight;
    int next = 0;
    for (;;) {
        std::vector<Request> batch;
        double est = 0.0;
        bool running = true;
        if ((int)inflight.size() < D) running = take_batch(s, inflight.empty(), &batch, &est);
        if (!batch.empty()) {
            BufSet& b = w->sets[next];
            b.reqs = std::move(batch);
            b.est_pairs = est;
            b.t_start = s->now();
            try {
                b.rc = launch_batch(w, b, b.reqs.data(), (int)b.reqs.size());
            } catch (...) {
                b.rc = GS_ERR_INTERNAL;
            }
            inflight.push_back(next);
            next = (next + 1) % D;
            continue;
        }
        if (!inflight.empty()) {
            BufSet& b = w->sets[inflight.front()];
            inflight.pop_front();
            settle(w, b, b.reqs.data(), (int)b.reqs.size(), b.rc, b.t_start, b.est_pairs);
            b.reqs.clear();
            continue;
        }
        if (!running) return;
    }
}

}  // namespace

extern "C" {

int gs_lod_select(const gs_lod_table* table, const gs_camera* cam, int64_t budget, int32_t* level, int64_t* total) {
    try {
        Lod t;
        int rc;
        if ((rc = copy_table(table, &t)) || (rc = check_camera(cam))) return rc;
        GS_REQUIRE(level && total, "NULL output");
        GS_REQUIRE(budget >= 0, "budget must be >= 0");
        return lod_select(t, *cam, budget, level, total);
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_lod_select");
    }
}

int gs_serve_create(const gs_gaussians* scene, const gs_lod_table* table, const gs_options* opt,
                    const gs_serve_config* cfg, int32_t device, gs_server** out) {
    gs_server* s = nullptr;
    try {
        GS_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        GS_REQUIRE(scene && scene->n >= 1 && scene->means && scene->scales && scene->quats && scene->opacities &&
                       scene->sh,
                   "scene is malformed");
        GS_REQUIRE(cfg != nullptr, "config is NULL");
        GS_REQUIRE(cfg->max_views_per_batch >= 1 && cfg->max_views_per_batch <= GS_MAX_VIEWS,
                   "max_views_per_batch outside 1..%d", GS_MAX_VIEWS);
        GS_REQUIRE(cfg->n_streams >= 1 && cfg->n_streams <= 8, "n_streams outside 1..8");
        GS_REQUIRE(cfg->slot_capacity >= 1 && cfg->slot_capacity <= 0xFFFFFF00LL, "slot_capacity out of range");
        GS_REQUIRE(cfg->pair_capacity >= 1 && cfg->pair_capacity <= 0xFFFFFF00LL, "pair_capacity out of range");
        GS_REQUIRE(cfg->pixel_capacity >= 256 && cfg->pixel_capacity <= (1LL << 31), "pixel_capacity out of range");
        GS_REQUIRE(cfg->queue_capacity >= 1, "queue_capacity must be >= 1");
        GS_REQUIRE(cfg->pipeline_depth >= 1 && cfg->pipeline_depth <= 4, "pipeline_depth outside 1..4");
        GS_REQUIRE(cfg->persistent_ctas >= 0 && cfg->persistent_ctas <= (1 << 20), "persistent_ctas out of range");
        GS_REQUIRE(std::isfinite(cfg->pairs_per_gaussian) && cfg->pairs_per_gaussian >= 0.0,
                   "pairs_per_gaussian must be finite and >= 0");
        GS_REQUIRE(((uintptr_t)scene->app & 15) == 0, "appearance offsets must be 16-byte aligned");
        s = new gs_server();
        int rc;
        if ((rc = copy_table(table, &s->lod)) || (rc = build_opt(opt, &s->opt))) {
            delete s;
            return rc;
        }
        for (size_t i = 0; i < s->lod.off.size(); ++i)
            if (s->lod.off[i] + s->lod.cnt[i] > scene->n) {
                delete s;
                return fail(GS_ERR_INVALID_ARG, "lod range %zu exceeds the scene's %lld Gaussians", i,
                            (long long)scene->n);
            }
        s->gp = GaussPtrs{scene->means, scene->scales, scene->quats, scene->opacities, scene->sh, scene->app};
        s->n = scene->n;
        s->cfg = *cfg;
        s->tile_cap = cfg->pixel_capacity / 16 + 1024;
        s->seg_cap = (int64_t)cfg->max_views_per_batch * s->lod.P;
        s->device = device;
        s->t0 = std::chrono::steady_clock::now();
        if (hipSetDevice(device) != hipSuccess) {
            delete s;
            return fail(GS_ERR_HIP, "hipSetDevice(%d) failed", device);
        }
        for (int i = 0; i < cfg->n_streams; ++i) {
            Worker* w = new Worker();
            w->srv = s;
            if ((rc = alloc_worker(s, w))) {
                free_worker(w);
                for (Worker* x : s->workers) free_worker(x);
                delete s;
                return rc;
            }
            s->workers.push_back(w);
        }
        for (Worker* w : s->workers) w->th = std::thread(worker_main, w);
        *out = s;
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_serve_create");
    }
}

double gs_serve_now(const gs_server* srv) { return srv ? srv->now() : 0.0; }

int gs_serve_submit(gs_server* s, const gs_camera* cam, int64_t budget, float* out_rgb, void* stream,
                    double t_arrival, uint64_t* ticket) {
    try {
        GS_REQUIRE(s != nullptr && out_rgb != nullptr && ticket != nullptr, "NULL argument");
        int rc = check_camera(cam);
        if (rc) return rc;
        GS_REQUIRE(budget >= 0, "budget must be >= 0");
        GS_REQUIRE(std::isfinite(t_arrival), "arrival time not finite");
        Request r;
        r.cam = *cam;
        r.budget = budget;
        r.out = out_rgb;
        r.t_arrival = t_arrival;
        r.level.assign(s->lod.P, 0);
        if ((rc = lod_select(s->lod, *cam, budget, r.level.data(), &r.n_sel))) return rc;
        r.n_pix = (int64_t)cam->width * cam->height;
        r.n_tiles = (int64_t)tiles_of(*cam);
        if (r.n_sel > s->cfg.slot_capacity || r.n_pix > s->cfg.pixel_capacity || r.n_tiles > s->tile_cap)
            return fail(GS_ERR_CAPACITY, "request exceeds one batch (%lld Gaussians, %lld pixels)",
                        (long long)r.n_sel, (long long)r.n_pix);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if ((int64_t)s->queue.size() >= s->cfg.queue_capacity) return fail(GS_EAGAIN, "queue full");
            if (!s->free_events.empty()) {
                r.ready = s->free_events.back();
                s->free_events.pop_back();
            }
        }
        // the ready event: recorded on the caller's stream, on the server's
        // device, so that the worker writes out_rgb after the caller's work
        int prev = 0;
        GS_HIP(hipGetDevice(&prev));
        hipError_t e = prev == s->device ? hipSuccess : hipSetDevice(s->device);
        if (e == hipSuccess && !r.ready) e = hipEventCreateWithFlags(&r.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r.ready, static_cast<hipStream_t>(stream));
        if (prev != s->device) (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            if (r.ready) recycle_events(s, &r, 1);
            return fail(GS_ERR_HIP, "recording the ready event failed: %s", hipGetErrorString(e));
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if ((int64_t)s->queue.size() >= s->cfg.queue_capacity) {
                s->free_events.push_back(r.ready);
                return fail(GS_EAGAIN, "queue full");
            }
            r.ticket = s->next_ticket++;
            *ticket = r.ticket;
            s->queue.push_back(std::move(r));
            s->submitted += 1;
        }
        s->cv.notify_all();
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_serve_submit");
    }
}

int gs_serve_poll(gs_server* s, gs_completion* done, int32_t max, int32_t timeout_us, int32_t* n_done) {
    try {
        GS_REQUIRE(s && done && n_done && max >= 1 && timeout_us >= 0, "bad arguments");
        std::unique_lock<std::mutex> lk(s->done_mu);
        s->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty(); });
        int k = 0;
        while (k < max && !s->done.empty()) {
            done[k++] = s->done.front();
            s->done.pop_front();
        }
        *n_done = k;
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_serve_poll");
    }
}

int gs_serve_stats_get(gs_server* s, gs_serve_stats* o) {
    try {
        GS_REQUIRE(s && o, "NULL argument");
        std::memset(o, 0, sizeof(*o));
        {
            std::lock_guard<std::mutex> lk(s->mu);
            o->submitted = s->submitted;
        }
        std::lock_guard<std::mutex> lk(s->done_mu);
        o->completed = s->completed;
        o->failed = s->failed;
        o->batches = s->batches;
        o->mean_batch_views = s->batches ? (double)s->batch_views / s->batches : 0.0;
        o->split_batches = s->split_batches;
        o->rebinned_batches = s->rebinned_batches;
        o->est_over_actual = s->est_batches ? s->est_over_actual / (double)s->est_batches : 0.0;
        if (!s->lat_ms.empty()) {
            std::vector<double> v = s->lat_ms;
            std::sort(v.begin(), v.end());
            // nearest-rank percentiles
            auto pct = [&](double q) {
                size_t k = (size_t)std::ceil(q * v.size());
                return v[std::min(v.size(), std::max<size_t>(k, 1)) - 1];
            };
            o->p50_ms = pct(0.50);
            o->p99_ms = pct(0.99);
            o->mean_ms = std::accumulate(v.begin(), v.end(), 0.0) / v.size();
            o->max_ms = v.back();
            o->span_s = s->last_done - s->first_arrival;
            if (o->span_s > 0.0) {
                o->req_per_s = s->completed / o->span_s;
                o->mpix_per_s = s->pixels / o->span_s * 1e-6;
            }
        }
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_serve_stats_get");
    }
}

int gs_serve_destroy(gs_server* s) {
    if (!s) return GS_OK;
    try {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv.notify_all();
        for (Worker* w : s->workers)
            if (w->th.joinable()) w->th.join();
        for (Worker* w : s->workers) free_worker(w);
        for (Request& r : s->queue)
            if (r.ready) (void)hipEventDestroy(r.ready);
        for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
        delete s;
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_serve_destroy");
    }
}

}  // extern "C"
