// C ABI of the rasterizer (declared in include/gs.h): argument checks,
// per-view constant tables, workspace layout and the launch sequence of
// each stage.  No call here allocates device memory.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <mutex>
#include <utility>
#include <vector>
#include <cstdio>
#include <algorithm>
#include <cstring>

#include "gs.h"
#include "gs_internal.h"
#include "host.h"

namespace gs {

namespace {
// event pairs recorded around timed launches, per timed kernel
std::atomic<bool> g_timing{false};
std::mutex g_timer_mu;
struct TimerPool {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
};
TimerPool g_timers[GS_KERNEL_TIMED];
}  // namespace

hipEvent_t timer_begin(int kernel, hipStream_t s) {
    if (!g_timing.load(std::memory_order_relaxed) || kernel < 0 || kernel >= GS_KERNEL_TIMED) return nullptr;
    std::lock_guard<std::mutex> lk(g_timer_mu);
    TimerPool& p = g_timers[kernel];
    if (p.used == p.ev.size()) {
        hipEvent_t b = nullptr, e = nullptr;
        if (hipEventCreate(&b) != hipSuccess) return nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipEventDestroy(b);
            return nullptr;
        }
        p.ev.emplace_back(b, e);
    }
    auto& pr = p.ev[p.used];
    if (hipEventRecord(pr.first, s) != hipSuccess) return nullptr;
    ++p.used;
    return pr.second;
}

void timer_end(hipEvent_t closing, hipStream_t s) {
    if (!closing) return;
    // the pool may have been released (timing disabled from another thread)
    // since timer_begin handed the event out
    std::lock_guard<std::mutex> lk(g_timer_mu);
    for (const auto& p : g_timers)
        for (size_t i = 0; i < p.used && i < p.ev.size(); ++i)
            if (p.ev[i].second == closing) {
                (void)hipEventRecord(closing, s);
                return;
            }
}

namespace host {

namespace {
thread_local char g_err[512] = "";
}  // namespace

const char* last_error() { return g_err; }

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int build_views(const gs_camera* cams, int32_t n_views, ViewTable* vt) {
    GS_REQUIRE(cams != nullptr, "cams is NULL");
    GS_REQUIRE(n_views >= 1 && n_views <= GS_MAX_VIEWS, "n_views=%d outside 1..%d", n_views, GS_MAX_VIEWS);
    std::memset(vt, 0, sizeof(*vt));
    int64_t tile_off = 0, pix_off = 0;
    for (int v = 0; v < n_views; ++v) {
        const gs_camera& c = cams[v];
        GS_REQUIRE(c.width >= 1 && c.width <= 16384 && c.height >= 1 && c.height <= 16384,
                   "view %d: image %dx%d outside 1..16384", v, c.width, c.height);
        GS_REQUIRE(std::isfinite(c.fx) && std::isfinite(c.fy) && c.fx > 0.0f && c.fy > 0.0f,
                   "view %d: focal lengths must be positive", v);
        GS_REQUIRE(std::isfinite(c.cx) && std::isfinite(c.cy), "view %d: principal point not finite", v);
        GS_REQUIRE(c.near_plane > 0.0f && c.far_plane > c.near_plane, "view %d: need 0 < near < far", v);
        for (int i = 0; i < 16; ++i) GS_REQUIRE(std::isfinite(c.viewmat[i]), "view %d: viewmat not finite", v);
        ViewK& V = vt->v[v];
        for (int r = 0; r < 3; ++r) {
            for (int k = 0; k < 3; ++k) V.R[3 * r + k] = c.viewmat[4 * r + k];
            V.t[r] = c.viewmat[4 * r + 3];
        }
        for (int i = 0; i < 3; ++i)
            V.campos[i] = -((double)V.R[i] * V.t[0] + (double)V.R[3 + i] * V.t[1] + (double)V.R[6 + i] * V.t[2]);
        V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy;
        V.znear = c.near_plane; V.zfar = c.far_plane;
        const double W = c.width, H = c.height, cx = c.cx, cy = c.cy, fx = c.fx, fy = c.fy;
        V.ulo = -(cx + 0.15 * W) / fx;
        V.uhi = (W - cx + 0.15 * W) / fx;
        V.vlo = -(cy + 0.15 * H) / fy;
        V.vhi = (H - cy + 0.15 * H) / fy;
        V.W = c.width; V.H = c.height;
        V.tiles_x = (c.width + kTile - 1) / kTile;
        V.tiles_y = (c.height + kTile - 1) / kTile;
        V.tile_off = (int32_t)tile_off;
        V.pix_off = pix_off;
        tile_off += (int64_t)V.tiles_x * V.tiles_y;
        pix_off += (int64_t)c.width * c.height;
    }
    GS_REQUIRE(tile_off < (1LL << 30), "too many tiles (%lld)", (long long)tile_off);
    vt->n_views = n_views;
    vt->total_tiles = (int32_t)tile_off;
    return GS_OK;
}

int build_opt(const gs_options* o, OptK* k) {
    GS_REQUIRE(o != nullptr, "options is NULL");
    GS_REQUIRE(o->sh_degree >= 0 && o->sh_degree <= 3, "sh_degree=%d outside 0..3", o->sh_degree);
    GS_REQUIRE(std::isfinite(o->dilation) && o->dilation >= 0.0f, "dilation must be >= 0");
    k->sh_degree = o->sh_degree;
    k->dilation = o->dilation;
    k->aa = o->aa_compensate ? 1 : 0;
    for (int i = 0; i < 3; ++i) k->bg[i] = o->bg[i];
    return GS_OK;
}

namespace {

int check_gaussians(const gs_gaussians* g, int32_t n_views) {
    GS_REQUIRE(g != nullptr, "gaussians is NULL");
    GS_REQUIRE(g->n >= 1, "n=%lld must be >= 1", (long long)g->n);
    GS_REQUIRE(g->means && g->scales && g->quats && g->opacities && g->sh, "a Gaussian parameter pointer is NULL");
    GS_REQUIRE(g->n * (int64_t)n_views <= 0xFFFFFF00LL, "n * n_views = %lld exceeds 32-bit slot ids",
               (long long)(g->n * n_views));
    GS_REQUIRE(((uintptr_t)g->app & 15) == 0, "appearance offsets must be 16-byte aligned");
    return GS_OK;
}

GaussPtrs gauss_ptrs(const gs_gaussians* g) {
    return GaussPtrs{g->means, g->scales, g->quats, g->opacities, g->sh, g->app};
}

// the offsets' gradient is produced only when the offsets are in use
GradPtrs grad_ptrs(const gs_gaussians* g, const gs_gaussians_grad* out) {
    return GradPtrs{out->d_means, out->d_scales, out->d_quats, out->d_opacities, out->d_sh,
                    g->app ? out->d_app : nullptr};
}

int check_proj(const gs_projected* p) {
    GS_REQUIRE(p != nullptr && p->rec && p->rect && p->tiles && p->depth_key, "projected buffers missing");
    GS_REQUIRE(((uintptr_t)p->tile_mask & 7) == 0, "tile_mask must be 8-byte aligned");
    return GS_OK;
}

Projected to_proj(const gs_projected* p) {
    return Projected{reinterpret_cast<float4*>(p->rec), reinterpret_cast<uint2*>(p->rect), p->tiles, p->depth_key,
                     p->tile_order, p->tile_mask};
}

int tile_bits(int64_t n_tiles) {
    int b = 0;
    while ((1LL << b) < n_tiles) ++b;
    return b;
}

constexpr int kTotals = 16 + 16 * kBinPairParts;

struct BinWs {
    uint32_t *dkeys, *dvals, *dkeys_alt, *dvals_alt;
    uint4* desc;
    uint32_t *tiles_s, *offsets;
    uint2* rect_s;
    uint64_t* mask_s;
    uint32_t* slot_s;
    uint32_t* hist;
    uint32_t* scan_tmp;
    unsigned long long* total;
    uint32_t* cnt;          // effective visible and pair counts on the device
    uint32_t *pkeys, *pkeys_alt, *pvals_alt;
};

size_t bin_layout(int64_t n_slots, int64_t cap, void* base, BinWs* w) {
    Carver c(base);
    const size_t N = (size_t)n_slots, Pc = (size_t)(cap > 0 ? cap : 1);
    w->dkeys = c.take<uint32_t>(N);
    w->dvals = c.take<uint32_t>(N);
    w->dkeys_alt = c.take<uint32_t>(N);
    w->dvals_alt = c.take<uint32_t>(N);
    w->desc = c.take<uint4>(2 * N);
    w->tiles_s = c.take<uint32_t>(N);
    w->offsets = c.take<uint32_t>(N);
    w->rect_s = c.take<uint2>(N);
    w->mask_s = c.take<uint64_t>(N);
    w->slot_s = c.take<uint32_t>(N);
    w->hist = c.take<uint32_t>(radix_hist_elems((uint32_t)(N > Pc ? N : Pc)));
    w->scan_tmp = c.take<uint32_t>(scan_tmp_elems((uint32_t)N));
    w->total = c.take<unsigned long long>(kTotals);   // [0] visible, [8] offsets total, [16 + 16k] pair parts
    w->cnt = c.take<uint32_t>(4);
    w->pkeys = c.take<uint32_t>(Pc);
    w->pkeys_alt = c.take<uint32_t>(Pc);
    w->pvals_alt = c.take<uint32_t>(Pc);
    return c.off;
}

}  // namespace

// segment area: work_off [T + 1] | state_off [T + 1] | stop_seg [T][256] |
// states [capacity][kSegFields][256]
size_t seg_fixed_bytes(int64_t n_tiles) {
    Carver c(nullptr);
    c.take<uint32_t>((size_t)n_tiles + 1);
    c.take<uint32_t>((size_t)n_tiles + 1);
    c.take<int32_t>((size_t)n_tiles * 256);
    return c.off;
}

constexpr size_t kSegStateBytes = (size_t)kSegFields * 256 * sizeof(float);

// a plan over `base` (NULL or too small: no segments)
void seg_layout(void* base, size_t bytes, int64_t n_tiles, SegPlan* plan, uint32_t* capacity) {
    *plan = SegPlan{nullptr, nullptr, nullptr, (uint32_t)n_tiles, nullptr, 0u};
    *capacity = 0;
    const size_t fixed = seg_fixed_bytes(n_tiles);
    if (!base || bytes < fixed) return;
    Carver c(base);
    plan->work_off = c.take<uint32_t>((size_t)n_tiles + 1);
    plan->state_off = c.take<uint32_t>((size_t)n_tiles + 1);
    plan->stop_seg = c.take<int32_t>((size_t)n_tiles * 256);
    plan->state = reinterpret_cast<float*>(static_cast<char*>(base) + fixed);
    *capacity = (uint32_t)std::min<size_t>((bytes - fixed) / kSegStateBytes, 1u << 24);
    plan->capacity = *capacity;
}

size_t bin_workspace_bytes(int64_t n_slots, int64_t pair_capacity) {
    if (n_slots < 1) n_slots = 1;
    BinWs w;
    return bin_layout(n_slots, pair_capacity, nullptr, &w);
}

int bin_sort_slots(const Projected& pr, const ViewTable& vt, int64_t n_slots, int64_t pair_capacity,
                   uint32_t* pair_vals, uint32_t* tile_ranges, int64_t* n_pairs_dev, void* ws, size_t ws_bytes,
                   hipStream_t s) {
    GS_REQUIRE(n_slots >= 1 && n_slots <= 0xFFFFFF00LL, "bad slot count %lld", (long long)n_slots);
    GS_REQUIRE(pair_vals && tile_ranges && n_pairs_dev && ws, "NULL output or workspace");
    GS_REQUIRE(pair_capacity >= 0 && pair_capacity <= 0xFFFFFF00LL, "pair_capacity out of range");
    GS_REQUIRE(((uintptr_t)ws & (kAlign - 1)) == 0, "workspace must be 256-byte aligned");
    GS_REQUIRE(((uintptr_t)n_pairs_dev & 7) == 0, "n_pairs must be 8-byte aligned");
    BinWs w;
    const size_t need = bin_layout(n_slots, pair_capacity, ws, &w);
    GS_REQUIRE(ws_bytes >= need, "workspace too small: %zu < %zu", ws_bytes, need);
    const uint32_t N = (uint32_t)n_slots, Pc = (uint32_t)pair_capacity;
    const hipEvent_t timed = timer_begin(GS_KERNEL_BIN_SORT, s);

    // 1. visible slots in slot order (scan of tiles > 0, scatter) with the
    //    pair count summed in the same pass; the counts stay on the device:
    //    every later launch is sized by N or the pair capacity and reads
    //    them there
    GS_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.total), 0u, 2 * kTotals, s));
    GS_HIP(exclusive_scan_nonzero_u32(pr.tiles, w.offsets, N, w.scan_tmp, w.total, w.total + 16, s));
    GS_HIP(launch_bin_counts(w.total, w.total + 16, Pc, n_pairs_dev, w.cnt, s));
    GS_HIP(launch_compact_visible(pr, w.offsets, N, w.dkeys, w.dvals, w.desc, s));
    // 2. depth order of the visible slots (stable: ties stay in slot order,
    //    which is compaction order); per depth rank its tile count, rectangle,
    //    mask and slot; exclusive scan -> pair offsets.  A visible slot emits
    //    at least one pair, so within the pair capacity there are at most
    //    min(N, capacity) of them (beyond it the counts read 0): the launches
    //    over visible slots are sized by that bound
    const uint32_t Nv = (uint32_t)std::min<int64_t>(n_slots, std::max<int64_t>(pair_capacity, 1));
    bool alt = false;
    GS_HIP(radix_sort_pairs(w.dkeys, w.dvals, w.dkeys_alt, w.dvals_alt, Nv, 0, 32, w.hist, s, &alt, w.cnt,
                            /*small_tiles=*/true));
    const uint32_t* sorted_pos = alt ? w.dvals_alt : w.dvals;
    GS_HIP(launch_gather_sorted(sorted_pos, w.desc, Nv, w.cnt, w.tiles_s, w.rect_s, w.mask_s, w.slot_s, s));
    GS_HIP(exclusive_scan_u32(w.tiles_s, w.offsets, Nv, w.scan_tmp, w.total + 8, s, w.cnt));
    // 3. expand into (tile, slot) pairs in depth order, then stable sort by tile id
    const int bits = tile_bits(vt.total_tiles);
    const int passes = radix_passes(Pc, 0, bits);
    uint32_t* vals_primary = (passes % 2 == 0) ? pair_vals : w.pvals_alt;
    uint32_t* vals_alt = (passes % 2 == 0) ? w.pvals_alt : pair_vals;
    GS_HIP(launch_emit_pairs(w.offsets, w.rect_s, pr.tile_mask ? w.mask_s : nullptr, w.slot_s, Nv, Pc, w.cnt, w.pkeys,
                             vals_primary, s));
    bool palt = false;
    GS_HIP(radix_sort_pairs(w.pkeys, vals_primary, w.pkeys_alt, vals_alt, Pc, 0, bits, w.hist, s, &palt, w.cnt + 1));
    const uint32_t* sorted_keys = palt ? w.pkeys_alt : w.pkeys;
    if ((palt ? vals_alt : vals_primary) != pair_vals)
        return fail(GS_ERR_INTERNAL, "tile sort ended in the wrong buffer");
    // 4. [start, end) per tile, and the compositing launch order
    GS_HIP(launch_tile_ranges(sorted_keys, Pc, w.cnt, tile_ranges, (uint32_t)vt.total_tiles, s));
    if (pr.tile_order) GS_HIP(launch_tile_order(tile_ranges, (uint32_t)vt.total_tiles, pr.tile_order, s));
    timer_end(timed, s);
    return GS_OK;
}

}  // namespace host
}  // namespace gs

using namespace gs;
using namespace gs::host;

extern "C" {

const char* gs_last_error(void) { return last_error(); }

const char* gs_version(void) { return "gsmi-rasterizer 0.1 (gfx950)"; }

int gs_kernel_timing(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    for (auto& p : g_timers) {
        p.used = 0;
        if (!enable) {
            // disabling releases the pool: the runtime stalls now and then
            // when many recorded events stay alive
            for (auto& pr : p.ev) {
                (void)hipEventSynchronize(pr.second);
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
            p.ev.clear();
        }
    }
    g_timing.store(enable != 0);
    return GS_OK;
}

int gs_kernel_timing_read(int32_t kernel, double* total_ms, int64_t* launches) {
    try {
        GS_REQUIRE(kernel >= 0 && kernel < GS_KERNEL_TIMED, "kernel id %d outside 0..%d", kernel, GS_KERNEL_TIMED - 1);
        GS_REQUIRE(total_ms && launches, "NULL output");
        std::lock_guard<std::mutex> lk(g_timer_mu);
        TimerPool& p = g_timers[kernel];
        double sum = 0.0;
        for (size_t i = 0; i < p.used; ++i) {
            float ms = 0.0f;
            GS_HIP(hipEventSynchronize(p.ev[i].second));
            GS_HIP(hipEventElapsedTime(&ms, p.ev[i].first, p.ev[i].second));
            sum += ms;
        }
        *total_ms = sum;
        *launches = (int64_t)p.used;
        p.used = 0;
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_kernel_timing_read");
    }
}

int gs_views_extent(const gs_camera* cams, int32_t n_views, int64_t* n_tiles, int64_t* n_pixels) {
    ViewTable vt;
    int rc = build_views(cams, n_views, &vt);
    if (rc) return rc;
    int64_t pix = 0;
    for (int v = 0; v < n_views; ++v) pix += (int64_t)cams[v].width * cams[v].height;
    if (n_tiles) *n_tiles = vt.total_tiles;
    if (n_pixels) *n_pixels = pix;
    return GS_OK;
}

int gs_project(const gs_gaussians* g, const gs_camera* cams, int32_t n_views, const gs_options* opt,
               const gs_projected* out, void* stream) {
    try {
        ViewTable vt;
        OptK ok;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = build_opt(opt, &ok)) ||
            (rc = check_gaussians(g, n_views)) || (rc = check_proj(out)))
            return rc;
        GaussPtrs gp = gauss_ptrs(g);
        GS_HIP(launch_project_fwd(gp, g->n, vt, ok, to_proj(out), (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_project");
    }
}

size_t gs_bin_workspace_size(int64_t n_slots, int64_t pair_capacity) {
    return bin_workspace_bytes(n_slots, pair_capacity);
}

int gs_bin_sort(const gs_projected* proj, const gs_camera* cams, int32_t n_views, int64_t n, int64_t pair_capacity,
                uint32_t* pair_vals, uint32_t* tile_ranges, int64_t* n_pairs_dev, void* ws, size_t ws_bytes,
                void* stream) {
    try {
        ViewTable vt;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = check_proj(proj))) return rc;
        GS_REQUIRE(n >= 1 && n * (int64_t)n_views <= 0xFFFFFF00LL, "bad n=%lld", (long long)n);
        return bin_sort_slots(to_proj(proj), vt, n * n_views, pair_capacity, pair_vals, tile_ranges, n_pairs_dev, ws,
                              ws_bytes, (hipStream_t)stream);
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_bin_sort");
    }
}

int gs_render_fwd(const gs_projected* proj, const uint32_t* pair_vals, const uint32_t* tile_ranges,
                  const gs_camera* cams, int32_t n_views, const gs_options* opt, float* rgb, float* depth,
                  float* alpha, float* T_final, int32_t* last, void* stream) {
    try {
        ViewTable vt;
        OptK ok;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = build_opt(opt, &ok)) || (rc = check_proj(proj)))
            return rc;
        GS_REQUIRE(pair_vals && tile_ranges && rgb && depth && alpha && T_final && last, "NULL buffer");
        GS_HIP(launch_render_fwd(to_proj(proj), pair_vals, reinterpret_cast<const uint2*>(tile_ranges), vt, ok, rgb,
                                 depth, alpha, T_final, last, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_render_fwd");
    }
}

int gs_render_count(const gs_projected* proj, const uint32_t* pair_vals, const uint32_t* tile_ranges,
                    const gs_camera* cams, int32_t n_views, int32_t* n_eval, void* stream) {
    try {
        ViewTable vt;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = check_proj(proj))) return rc;
        GS_REQUIRE(pair_vals && tile_ranges && n_eval, "NULL buffer");
        GS_HIP(launch_render_count(to_proj(proj), pair_vals, reinterpret_cast<const uint2*>(tile_ranges), vt, n_eval,
                                   (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_render_count");
    }
}

size_t gs_loss_workspace_size(int64_t n_pix) {
    if (n_pix < 1) n_pix = 1;
    return align_up(loss_partials(n_pix) * sizeof(double));
}

int gs_loss_l1_depth(const float* rgb, const float* depth, const float* alpha, const float* target_rgb,
                     const float* target_depth, int64_t n_pix, float lambda_depth, float* loss, float* d_rgb,
                     float* d_depth, float* d_alpha, void* ws, size_t ws_bytes, void* stream) {
    try {
        GS_REQUIRE(n_pix >= 1 && n_pix <= (1LL << 34), "n_pix=%lld out of range", (long long)n_pix);
        GS_REQUIRE(rgb && target_rgb && loss && d_rgb && d_depth && d_alpha && ws, "NULL buffer");
        GS_REQUIRE(!target_depth || (depth && alpha), "the depth term needs depth and alpha");
        GS_REQUIRE(std::isfinite(lambda_depth), "lambda_depth not finite");
        GS_REQUIRE(((uintptr_t)ws & 7) == 0, "workspace must be 8-byte aligned");
        GS_REQUIRE(ws_bytes >= gs_loss_workspace_size(n_pix), "workspace too small");
        GS_HIP(launch_loss(rgb, depth, alpha, target_rgb, target_depth, n_pix, lambda_depth, loss, d_rgb, d_depth,
                           d_alpha, static_cast<double*>(ws), (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_loss_l1_depth");
    }
}

int gs_loss_l1_depth_noalloc(const float* rgb, const float* depth, const float* alpha, const float* target_rgb,
                             const float* target_depth, int64_t n_pix, float lambda_depth, float* loss, float* d_rgb,
                             float* d_depth, float* d_alpha, void* stream) {
    try {
        GS_REQUIRE(n_pix >= 1, "n_pix=%lld out of range", (long long)n_pix);
        if (n_pix > loss_scratch_max_pixels())
            return fail(GS_ERR_CAPACITY, "n_pix=%lld exceeds the %lld pixels of the static scratch", (long long)n_pix,
                        (long long)loss_scratch_max_pixels());
        GS_REQUIRE(rgb && target_rgb && loss && d_rgb && d_depth && d_alpha, "NULL buffer");
        GS_REQUIRE(!target_depth || (depth && alpha), "the depth term needs depth and alpha");
        GS_REQUIRE(std::isfinite(lambda_depth), "lambda_depth not finite");
        double* scratch = nullptr;
        GS_HIP(loss_scratch_ptr(&scratch));
        GS_HIP(launch_loss(rgb, depth, alpha, target_rgb, target_depth, n_pix, lambda_depth, loss, d_rgb, d_depth,
                           d_alpha, scratch, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_loss_l1_depth_noalloc");
    }
}

size_t gs_dssim_workspace_size(int32_t width, int32_t height) {
    if (width < 1 || height < 1) return 0;
    Carver c(nullptr);
    for (int i = 0; i < 3; ++i) c.take<float>((size_t)width * height * 3);
    c.take<double>(ssim_partials(width, height));
    return c.off;
}

int gs_dssim(const float* rgb, const float* target, int32_t width, int32_t height, float weight, float* loss,
             float* d_rgb, void* ws, size_t ws_bytes, void* stream) {
    try {
        GS_REQUIRE(width >= 1 && width <= 16384 && height >= 1 && height <= 16384, "image %dx%d outside 1..16384",
                   width, height);
        GS_REQUIRE(rgb && target && loss && d_rgb && ws, "NULL buffer");
        GS_REQUIRE(std::isfinite(weight), "weight not finite");
        GS_REQUIRE(((uintptr_t)ws & (kAlign - 1)) == 0, "workspace must be 256-byte aligned");
        GS_REQUIRE(ws_bytes >= gs_dssim_workspace_size(width, height), "workspace too small");
        Carver c(ws);
        float* Pa = c.take<float>((size_t)width * height * 3);
        float* Pb = c.take<float>((size_t)width * height * 3);
        float* Pc = c.take<float>((size_t)width * height * 3);
        double* partial = c.take<double>(ssim_partials(width, height));
        GS_HIP(launch_dssim(rgb, target, width, height, weight, loss, d_rgb, Pa, Pb, Pc, partial, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_dssim");
    }
}

size_t gs_render_bwd_workspace_size(int64_t n_slots) {
    if (n_slots < 1) n_slots = 1;
    return align_up((size_t)n_slots * GS_GRAD2D_FLOATS * sizeof(float));
}

const float* gs_render_bwd_grad2d(void* ws) { return static_cast<const float*>(ws); }


size_t gs_seg_workspace_size(int64_t n_tiles, int64_t n_pairs) {
    if (n_tiles < 1) n_tiles = 1;
    if (n_pairs < 0) n_pairs = 0;
    return seg_fixed_bytes(n_tiles) + ((size_t)n_pairs / kSegLen + 1) * kSegStateBytes;
}

int gs_render_fwd_seg(const gs_projected* proj, const uint32_t* pair_vals, const uint32_t* tile_ranges,
                      const gs_camera* cams, int32_t n_views, const gs_options* opt, float* rgb, float* depth,
                      float* alpha, float* T_final, int32_t* last, void* seg_ws, size_t seg_ws_bytes,
                      void* stream) {
    try {
        ViewTable vt;
        OptK ok;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = build_opt(opt, &ok)) || (rc = check_proj(proj)))
            return rc;
        GS_REQUIRE(pair_vals && tile_ranges && rgb && depth && alpha && T_final && last, "NULL buffer");
        GS_REQUIRE(((uintptr_t)seg_ws & (kAlign - 1)) == 0, "segment workspace must be 256-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        SegPlan plan;
        uint32_t cap;
        seg_layout(seg_ws, seg_ws_bytes, vt.total_tiles, &plan, &cap);
        const Projected pr = to_proj(proj);
        const uint2* rg = reinterpret_cast<const uint2*>(tile_ranges);
        if (plan.work_off) GS_HIP(launch_seg_plan(pr, rg, vt, cap, plan, s));
        GS_HIP(launch_render_fwd(pr, pair_vals, rg, vt, ok, rgb, depth, alpha, T_final, last, s, 0, nullptr,
                                 plan.work_off ? &plan : nullptr));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_render_fwd_seg");
    }
}

int gs_render_bwd(const gs_gaussians* g, const gs_camera* cams, int32_t n_views, const gs_options* opt,
                  const gs_projected* proj, const uint32_t* pair_vals, const uint32_t* tile_ranges,
                  const float* T_final, const int32_t* last, const float* d_rgb, const float* d_depth,
                  const float* d_alpha, const gs_gaussians_grad* out, float* mean2d_grad_norm, float* absgrad,
                  void* ws, size_t ws_bytes, void* stream) {
    try {
        ViewTable vt;
        OptK ok;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = build_opt(opt, &ok)) ||
            (rc = check_gaussians(g, n_views)) || (rc = check_proj(proj)))
            return rc;
        GS_REQUIRE(pair_vals && tile_ranges && T_final && last && out && mean2d_grad_norm && ws, "NULL buffer");
        GS_REQUIRE(out->d_means && out->d_scales && out->d_quats && out->d_opacities && out->d_sh,
                   "NULL gradient output");
        const int64_t n_slots = g->n * n_views;
        const size_t g2_bytes = gs_render_bwd_workspace_size(n_slots);
        GS_REQUIRE(ws_bytes >= g2_bytes, "workspace too small");
        GS_REQUIRE(((uintptr_t)ws & (kAlign - 1)) == 0, "workspace must be 256-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        float* grad2d = static_cast<float*>(ws);
        SegPlan plan;
        uint32_t cap;
        seg_layout(static_cast<char*>(ws) + g2_bytes, ws_bytes - g2_bytes, vt.total_tiles, &plan, &cap);
        GS_HIP(zero_seen_grad2d(proj->tiles, grad2d, n_slots, s));
        const Projected pr = to_proj(proj);
        const uint2* rg = reinterpret_cast<const uint2*>(tile_ranges);
        if (plan.work_off) GS_HIP(launch_seg_prepare(pr, pair_vals, rg, vt, last, cap, plan, s));
        GS_HIP(launch_render_bwd(pr, pair_vals, rg, vt, ok, T_final, last, d_rgb, d_depth, d_alpha, grad2d, plan, cap,
                                 absgrad != nullptr, s));
        GaussPtrs gp = gauss_ptrs(g);
        GradPtrs go = grad_ptrs(g, out);
        GS_REQUIRE(((uintptr_t)go.app & 15) == 0, "d_app must be 16-byte aligned");
        GS_HIP(launch_project_bwd(gp, g->n, vt, ok, pr, grad2d, go, mean2d_grad_norm, absgrad, s));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_render_bwd");
    }
}

int gs_composite_bwd(const gs_projected* proj, const uint32_t* pair_vals, const uint32_t* tile_ranges,
                     const gs_camera* cams, int32_t n_views, const gs_options* opt, const float* T_final,
                     const int32_t* last, const float* d_rgb, const float* d_depth, const float* d_alpha,
                     int32_t abs_sums, int64_t n_slots, float* grad2d, void* seg_ws, size_t seg_ws_bytes,
                     int32_t seg_ready, void* stream) {
    try {
        ViewTable vt;
        OptK ok;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = build_opt(opt, &ok)) || (rc = check_proj(proj)))
            return rc;
        GS_REQUIRE(pair_vals && tile_ranges && T_final && last && grad2d, "NULL buffer");
        GS_REQUIRE(n_slots >= 1 && n_slots <= 0xFFFFFF00LL, "bad n_slots");
        GS_REQUIRE(((uintptr_t)seg_ws & (kAlign - 1)) == 0, "segment workspace must be 256-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        SegPlan plan;
        uint32_t cap;
        seg_layout(seg_ws, seg_ws_bytes, vt.total_tiles, &plan, &cap);
        GS_HIP(zero_seen_grad2d(proj->tiles, grad2d, n_slots, s));
        const Projected pr = to_proj(proj);
        const uint2* rg = reinterpret_cast<const uint2*>(tile_ranges);
        // seg_ready: the plan and the states are those gs_render_fwd_seg wrote
        if (plan.work_off && !seg_ready) GS_HIP(launch_seg_prepare(pr, pair_vals, rg, vt, last, cap, plan, s));
        GS_HIP(launch_render_bwd(pr, pair_vals, rg, vt, ok, T_final, last, d_rgb, d_depth, d_alpha, grad2d, plan, cap,
                                 abs_sums != 0, s));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_composite_bwd");
    }
}

int gs_grads_zero(const gs_gaussians_grad* out, int64_t n, void* stream) {
    try {
        GS_REQUIRE(out && out->d_means && out->d_scales && out->d_quats && out->d_opacities && out->d_sh,
                   "NULL gradient output");
        GS_REQUIRE(n >= 0, "n=%lld must be >= 0", (long long)n);
        const GradPtrs go{out->d_means, out->d_scales, out->d_quats, out->d_opacities, out->d_sh, out->d_app};
        GS_HIP(launch_zero_grads(go, n, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_grads_zero");
    }
}

int gs_project_bwd(const gs_gaussians* g, const gs_camera* cams, int32_t n_views, const gs_options* opt,
                   const gs_projected* proj, const float* grad2d, const gs_gaussians_grad* out,
                   float* mean2d_grad_norm, float* absgrad, int32_t grads_zeroed, void* stream) {
    try {
        ViewTable vt;
        OptK ok;
        int rc;
        if ((rc = build_views(cams, n_views, &vt)) || (rc = build_opt(opt, &ok)) ||
            (rc = check_gaussians(g, n_views)) || (rc = check_proj(proj)))
            return rc;
        GS_REQUIRE(grad2d && out && mean2d_grad_norm, "NULL buffer");
        GS_REQUIRE(out->d_means && out->d_scales && out->d_quats && out->d_opacities && out->d_sh,
                   "NULL gradient output");
        GaussPtrs gp = gauss_ptrs(g);
        GradPtrs go = grad_ptrs(g, out);
        GS_REQUIRE(((uintptr_t)go.app & 15) == 0, "d_app must be 16-byte aligned");
        GS_HIP(launch_project_bwd(gp, g->n, vt, ok, to_proj(proj), grad2d, go, mean2d_grad_norm, absgrad,
                                  (hipStream_t)stream, grads_zeroed != 0));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_project_bwd");
    }
}

size_t gs_appearance_workspace_size(int64_t n) { return app_workspace_bytes(n < 0 ? 0 : n); }

int gs_appearance_fwd(const float* gauss_emb, int64_t n, const float* image_emb, const gs_appearance_mlp* mlp,
                      float reg_weight, float* offsets, float* reg_value, void* ws, size_t ws_bytes, void* stream) {
    try {
        GS_REQUIRE(n >= 0, "n=%lld must be >= 0", (long long)n);
        GS_REQUIRE(image_emb && mlp && mlp->w1 && mlp->b1 && mlp->w2 && mlp->b2 && ws, "NULL argument");
        GS_REQUIRE(n == 0 || (gauss_emb && offsets), "NULL embedding or offset buffer");
        GS_REQUIRE(((uintptr_t)gauss_emb & 15) == 0 && ((uintptr_t)offsets & 15) == 0,
                   "embeddings and offsets must be 16-byte aligned");
        GS_REQUIRE(ws_bytes >= app_workspace_bytes(n), "workspace too small");
        const AppMlp w{mlp->w1, mlp->b1, mlp->w2, mlp->b2};
        GS_HIP(launch_app_fwd(gauss_emb, n, image_emb, w, reg_weight, offsets, reg_value, ws, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_appearance_fwd");
    }
}

int gs_appearance_bwd(const float* gauss_emb, int64_t n, const float* image_emb, const gs_appearance_mlp* mlp,
                      const float* offsets, const float* d_offsets, const float* d_reg, float reg_weight,
                      float* d_gauss_emb, const gs_appearance_grad* out, void* ws, size_t ws_bytes, void* stream) {
    try {
        GS_REQUIRE(n >= 0, "n=%lld must be >= 0", (long long)n);
        GS_REQUIRE(image_emb && mlp && mlp->w1 && mlp->b1 && mlp->w2 && mlp->b2 && ws && out, "NULL argument");
        GS_REQUIRE(out->d_w1 && out->d_b1 && out->d_w2 && out->d_b2, "NULL weight gradient");
        GS_REQUIRE(n == 0 || (gauss_emb && offsets && d_offsets && d_gauss_emb), "NULL per-Gaussian buffer");
        GS_REQUIRE(((uintptr_t)gauss_emb & 15) == 0 && ((uintptr_t)d_gauss_emb & 15) == 0,
                   "embeddings and their gradient must be 16-byte aligned");
        GS_REQUIRE(ws_bytes >= app_workspace_bytes(n), "workspace too small");
        const AppMlp w{mlp->w1, mlp->b1, mlp->w2, mlp->b2};
        const AppGrad g{out->d_w1, out->d_b1, out->d_w2, out->d_b2, out->d_image_emb};
        GS_HIP(launch_app_bwd(gauss_emb, n, image_emb, w, offsets, d_offsets, d_reg, reg_weight, d_gauss_emb, g, ws,
                              (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_appearance_bwd");
    }
}

}  // extern "C"
