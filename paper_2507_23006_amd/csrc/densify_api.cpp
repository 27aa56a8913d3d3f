// C ABI of the densification bookkeeping and the 3D smoothing filter
// (kernels in densify.hip): argument checks, workspace carving and the
// launch sequence of the budgeted selection.
#include <cstring>

#include "host.h"

using namespace gs;
using namespace gs::host;

namespace {

struct DensWs {
    uint32_t *cand, *pos, *pruned, *ppos, *key, *ckey, *cidx, *ckey_alt, *cidx_alt, *hist, *scan_tmp;
    unsigned long long* total;   // [0] candidates, [8] pruned (separate 64-byte lines)
};

size_t dens_layout(int64_t n, void* base, DensWs* w) {
    const uint32_t N = (uint32_t)(n < 1 ? 1 : n);
    Carver c(base);
    w->cand = c.take<uint32_t>(N);
    w->pos = c.take<uint32_t>(N);
    w->pruned = c.take<uint32_t>(N);
    w->ppos = c.take<uint32_t>(N);
    w->key = c.take<uint32_t>(N);
    w->ckey = c.take<uint32_t>(N);
    w->cidx = c.take<uint32_t>(N);
    w->ckey_alt = c.take<uint32_t>(N);
    w->cidx_alt = c.take<uint32_t>(N);
    w->hist = c.take<uint32_t>(radix_hist_elems(N));
    w->scan_tmp = c.take<uint32_t>(scan_tmp_elems(N));
    w->total = c.take<unsigned long long>(16);
    return c.off;
}

unsigned long long* pinned_pair() {
    thread_local unsigned long long* p = nullptr;
    if (!p && hipHostMalloc(reinterpret_cast<void**>(&p), 16 * sizeof(unsigned long long), hipHostMallocDefault) !=
                  hipSuccess)
        p = nullptr;
    return p;
}

}  // namespace

extern "C" {

int gs_densify_accumulate(const uint32_t* tiles, const float* grad_norm, const float* absgrad, int32_t n_views,
                          int64_t n, const float* view_scale, float* accum, int32_t* count, void* stream) {
    try {
        GS_REQUIRE(n >= 1, "n=%lld must be >= 1", (long long)n);
        GS_REQUIRE(n_views >= 1 && n_views <= GS_MAX_VIEWS, "n_views=%d outside 1..%d", n_views, GS_MAX_VIEWS);
        GS_REQUIRE(n * (int64_t)n_views <= 0xFFFFFF00LL, "n * n_views exceeds 32-bit slot ids");
        GS_REQUIRE(tiles && accum && count, "NULL buffer");
        GS_REQUIRE((grad_norm != nullptr) != (absgrad != nullptr), "give exactly one of grad_norm and absgrad");
        GS_REQUIRE(((uintptr_t)absgrad & 7) == 0, "absgrad must be 8-byte aligned");
        DensViewScale sc;
        for (int v = 0; v < GS_MAX_VIEWS; ++v) sc.s[v] = (view_scale && v < n_views) ? view_scale[v] : 1.0f;
        GS_HIP(launch_dens_accumulate(tiles, grad_norm, absgrad, n_views, n, sc, accum, count, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_densify_accumulate");
    }
}

size_t gs_densify_workspace_size(int64_t n) {
    DensWs w;
    return dens_layout(n, nullptr, &w);
}

int gs_densify_select(const float* accum, const int32_t* count, const float* means, const float* scales,
                      const float* opacities, int64_t n, const gs_densify_params* p, uint8_t* action,
                      int64_t* counts, void* ws, size_t ws_bytes, void* stream) {
    try {
        GS_REQUIRE(n >= 1 && n <= 0xFFFFFF00LL, "n=%lld outside 1..2^32-256", (long long)n);
        GS_REQUIRE(accum && count && means && scales && opacities && p && action && counts && ws, "NULL argument");
        GS_REQUIRE(((uintptr_t)ws & (kAlign - 1)) == 0, "workspace must be 256-byte aligned");
        GS_REQUIRE(ws_bytes >= gs_densify_workspace_size(n), "workspace too small");
        GS_REQUIRE(p->d_max > 0.0f && p->eta >= 1.0f && p->tau_min > 0.0f, "need d_max > 0, eta >= 1, tau_min > 0");
        GS_REQUIRE(p->budget >= 0, "budget must be >= 0");
        for (int k = 0; k < 3; ++k) GS_REQUIRE(p->box_min[k] <= p->box_max[k], "empty partition box");
        hipStream_t s = (hipStream_t)stream;
        DensWs w;
        dens_layout(n, ws, &w);
        DensParams dp;
        for (int k = 0; k < 3; ++k) {
            dp.box_min[k] = p->box_min[k];
            dp.box_max[k] = p->box_max[k];
        }
        dp.tau_min = p->tau_min;
        dp.eta = p->eta;
        dp.d_max = p->d_max;
        dp.prune_opacity = p->prune_opacity;
        const uint32_t N = (uint32_t)n;
        GS_HIP(launch_dens_classify(accum, count, means, opacities, n, dp, action, w.cand, w.pruned, w.key, s));
        GS_HIP(exclusive_scan_u32(w.cand, w.pos, N, w.scan_tmp, w.total, s));
        GS_HIP(exclusive_scan_u32(w.pruned, w.ppos, N, w.scan_tmp, w.total + 8, s));
        unsigned long long* host = pinned_pair();
        if (!host) return fail(GS_ERR_HIP, "pinned host buffer unavailable");
        GS_HIP(hipMemcpyAsync(host, w.total, 16 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        GS_HIP(hipStreamSynchronize(s));
        const int64_t E = (int64_t)host[0], pruned = (int64_t)host[8];
        if (E > n || pruned > n) return fail(GS_ERR_INTERNAL, "inconsistent totals");
        int64_t K = p->budget - (n - pruned);
        if (K < 0) K = 0;
        const int64_t grown = K < E ? K : E;
        if (grown == E && E > 0) {
            GS_HIP(launch_dens_mark(nullptr, 0, w.cand, true, scales, n, p->split_scale, action, s));
        } else if (grown > 0) {
            GS_HIP(launch_dens_compact(w.cand, w.pos, w.key, n, w.ckey, w.cidx, s));
            bool alt = false;
            GS_HIP(radix_sort_pairs(w.ckey, w.cidx, w.ckey_alt, w.cidx_alt, (uint32_t)E, 0, 32, w.hist, s, &alt));
            GS_HIP(launch_dens_mark(alt ? w.cidx_alt : w.cidx, (uint32_t)grown, nullptr, false, scales, n,
                                    p->split_scale, action, s));
        }
        counts[0] = E;
        counts[1] = pruned;
        counts[2] = grown;
        counts[3] = K;
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_densify_select");
    }
}

int gs_filter3d_rate(const float* means, int64_t n, const gs_camera* cams, int32_t n_cams, float* rate,
                     void* stream) {
    try {
        GS_REQUIRE(n >= 1, "n=%lld must be >= 1", (long long)n);
        GS_REQUIRE(means && rate && cams, "NULL argument");
        GS_REQUIRE(n_cams >= 1, "need at least one camera");
        for (int32_t b = 0; b < n_cams; b += GS_MAX_VIEWS) {
            const int32_t m = n_cams - b < GS_MAX_VIEWS ? n_cams - b : GS_MAX_VIEWS;
            ViewTable vt;
            int rc = build_views(cams + b, m, &vt);
            if (rc) return rc;
            GS_HIP(launch_filter_rate(means, n, vt, b > 0, rate, (hipStream_t)stream));
        }
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_filter3d_rate");
    }
}

int gs_filter3d_fwd(const float* scales, const float* opacities, const float* rate, int64_t n, float s_f,
                    float* scales_out, float* opacities_out, void* stream) {
    try {
        GS_REQUIRE(n >= 1, "n=%lld must be >= 1", (long long)n);
        GS_REQUIRE(scales && opacities && rate && scales_out && opacities_out, "NULL argument");
        GS_REQUIRE(s_f >= 0.0f, "s_f must be >= 0");
        GS_HIP(launch_filter_fwd(scales, opacities, rate, n, s_f, scales_out, opacities_out, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_filter3d_fwd");
    }
}

int gs_filter3d_bwd(const float* scales, const float* opacities, const float* rate, int64_t n, float s_f,
                    const float* d_scales_out, const float* d_opacities_out, float* d_scales, float* d_opacities,
                    void* stream) {
    try {
        GS_REQUIRE(n >= 1, "n=%lld must be >= 1", (long long)n);
        GS_REQUIRE(scales && opacities && rate && d_scales_out && d_opacities_out && d_scales && d_opacities,
                   "NULL argument");
        GS_REQUIRE(s_f >= 0.0f, "s_f must be >= 0");
        GS_HIP(launch_filter_bwd(scales, opacities, rate, n, s_f, d_scales_out, d_opacities_out, d_scales,
                                 d_opacities, (hipStream_t)stream));
        return GS_OK;
    } catch (...) {
        return fail(GS_ERR_INTERNAL, "unexpected exception in gs_filter3d_bwd");
    }
}

}  // extern "C"
