// Densification bookkeeping and the 3D smoothing filter -- gfx950.
//
// Consumers of the backward's per-view statistics between training steps:
//   accumulate  per Gaussian, the views that rasterized it add their
//               |dL/d mean2d| (or the AbsGS per-axis absolute sums' length)
//               times a per-view scale to a running sum, and count;
//   classify    mean = sum / count against the in-partition threshold of
//               Eq. 4, tau_i = tau_min (min(d_i, d_max) / d_max (eta - 1) + 1)
//               with d_i the distance to the partition box; pruning by an
//               opacity floor; a sort key of mean / tau_i for the budget cap;
//   mark        the first K candidates of the key order are cloned or split
//               (by their largest scale);
//   filter      Mip-Splatting's 3D smoothing filter: the sampling rate
//               max f_x / depth over the cameras that hold the mean, and
//               scales sqrt(s^2 + (s_f / rate)^2) with the opacity scaled by
//               prod s / s' (forward and backward).
// All are one thread per Gaussian over structure-of-arrays streams: HBM-bound.
// Decisions compare FP64 values formed from the float32 inputs (the mean is
// a float32 division, as stored).
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kDT = 256;

__global__ __launch_bounds__(kDT) void k_dens_accumulate(const uint32_t* __restrict__ tiles,
                                                         const float* __restrict__ grad_norm,
                                                         const float2* __restrict__ absgrad, int32_t n_views,
                                                         int64_t n, DensViewScale sc, float* __restrict__ accum,
                                                         int32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * kDT + threadIdx.x;
    if (i >= n) return;
    float a = accum[i];
    int32_t c = count[i];
    for (int v = 0; v < n_views; ++v) {
        const int64_t slot = (int64_t)v * n + i;
        if (!tiles[slot]) continue;
        float val;
        if (absgrad) {
            const float2 g = absgrad[slot];
            val = sqrtf(g.x * g.x + g.y * g.y);
        } else {
            val = grad_norm[slot];
        }
        a += val * sc.s[v];
        c += 1;
    }
    accum[i] = a;
    count[i] = c;
}

__device__ __forceinline__ double box_dist(double x, double lo, double hi) {
    return fmax(fmax(lo - x, x - hi), 0.0);
}

// action: PRUNE or KEEP; cand[i] = 1 for candidates with key[i] = ~bits(mean / tau)
// (ascending keys = descending scores); pruned[i] = 1 for pruned Gaussians
__global__ __launch_bounds__(kDT) void k_dens_classify(const float* __restrict__ accum,
                                                       const int32_t* __restrict__ count,
                                                       const float* __restrict__ means,
                                                       const float* __restrict__ opac, int64_t n, DensParams p,
                                                       uint8_t* __restrict__ action, uint32_t* __restrict__ cand,
                                                       uint32_t* __restrict__ pruned, uint32_t* __restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * kDT + threadIdx.x;
    if (i >= n) return;
    const int32_t c = count[i];
    const float mean = c > 0 ? accum[i] / (float)c : 0.0f;
    const double dx = box_dist(means[i], p.box_min[0], p.box_max[0]);
    const double dy = box_dist(means[n + i], p.box_min[1], p.box_max[1]);
    const double dz = box_dist(means[2 * n + i], p.box_min[2], p.box_max[2]);
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double tau = (double)p.tau_min * (fmin(d, (double)p.d_max) / (double)p.d_max * ((double)p.eta - 1.0) + 1.0);
    const bool pr = opac[i] < p.prune_opacity;
    const bool cd = !pr && (double)mean > tau;
    action[i] = pr ? (uint8_t)GS_DENSIFY_PRUNE : (uint8_t)GS_DENSIFY_KEEP;
    cand[i] = cd ? 1u : 0u;
    pruned[i] = pr ? 1u : 0u;
    key[i] = cd ? ~__float_as_uint((float)((double)mean / tau)) : 0xFFFFFFFFu;
}

// candidates in index order: (key, index) at their scan position
__global__ __launch_bounds__(kDT) void k_dens_compact(const uint32_t* __restrict__ cand,
                                                      const uint32_t* __restrict__ pos,
                                                      const uint32_t* __restrict__ key, int64_t n,
                                                      uint32_t* __restrict__ ckey, uint32_t* __restrict__ cidx) {
    const int64_t i = (int64_t)blockIdx.x * kDT + threadIdx.x;
    if (i >= n || !cand[i]) return;
    ckey[pos[i]] = key[i];
    cidx[pos[i]] = (uint32_t)i;
}

__device__ __forceinline__ uint8_t grow_kind(const float* __restrict__ scales, int64_t n, int64_t i, float thr) {
    const float m = fmaxf(scales[i], fmaxf(scales[n + i], scales[2 * n + i]));
    return m > thr ? (uint8_t)GS_DENSIFY_SPLIT : (uint8_t)GS_DENSIFY_CLONE;
}

// the first k entries of the sorted candidate list grow
__global__ __launch_bounds__(kDT) void k_dens_mark_sorted(const uint32_t* __restrict__ sidx, uint32_t k,
                                                          const float* __restrict__ scales, int64_t n, float thr,
                                                          uint8_t* __restrict__ action) {
    const uint32_t r = blockIdx.x * kDT + threadIdx.x;
    if (r >= k) return;
    const int64_t i = sidx[r];
    action[i] = grow_kind(scales, n, i, thr);
}

// every candidate grows (the budget holds them all)
__global__ __launch_bounds__(kDT) void k_dens_mark_all(const uint32_t* __restrict__ cand,
                                                       const float* __restrict__ scales, int64_t n, float thr,
                                                       uint8_t* __restrict__ action) {
    const int64_t i = (int64_t)blockIdx.x * kDT + threadIdx.x;
    if (i >= n || !cand[i]) return;
    action[i] = grow_kind(scales, n, i, thr);
}

// rate = max(rate if `accumulate`, max over the table's views holding the mean of fx / depth)
__global__ __launch_bounds__(kDT) void k_filter_rate(const float* __restrict__ means, int64_t n, ViewTable vt,
                                                     int accumulate, float* __restrict__ rate) {
    const int64_t i = (int64_t)blockIdx.x * kDT + threadIdx.x;
    if (i >= n) return;
    const double m0 = means[i], m1 = means[n + i], m2 = means[2 * n + i];
    double best = 0.0;
    for (int v = 0; v < vt.n_views; ++v) {
        const ViewK& V = vt.v[v];
        const double tz = (double)V.R[6] * m0 + (double)V.R[7] * m1 + (double)V.R[8] * m2 + (double)V.t[2];
        if (!(tz >= (double)V.znear && tz <= (double)V.zfar)) continue;
        const double tx = (double)V.R[0] * m0 + (double)V.R[1] * m1 + (double)V.R[2] * m2 + (double)V.t[0];
        const double ty = (double)V.R[3] * m0 + (double)V.R[4] * m1 + (double)V.R[5] * m2 + (double)V.t[1];
        // x / z within [ulo, uhi] as products (z >= near > 0): one division per camera
        if (tx >= V.ulo * tz && tx <= V.uhi * tz && ty >= V.vlo * tz && ty <= V.vhi * tz)
            best = fmax(best, (double)V.fx / tz);
    }
    const float r = (float)best;
    rate[i] = accumulate ? fmaxf(rate[i], r) : r;
}

// filter variance (s_f / rate)^2, 0 for an unseen Gaussian
__device__ __forceinline__ double filter_var(float rate, float s_f) {
    if (!(rate > 0.0f)) return 0.0;
    const double q = (double)s_f / (double)rate;
    return q * q;
}

__global__ __launch_bounds__(kDT) void k_filter_fwd(const float* __restrict__ scales, const float* __restrict__ opac,
                                                    const float* __restrict__ rate, int64_t n, float s_f,
                                                    float* __restrict__ scales_out, float* __restrict__ opac_out) {
    const int64_t i = (int64_t)blockIdx.x * kDT + threadIdx.x;
    if (i >= n) return;
    const double var = filter_var(rate[i], s_f);
    double comp = 1.0;
    for (int k = 0; k < 3; ++k) {
        const double s = scales[k * n + i];
        const double s2 = sqrt(s * s + var);
        scales_out[k * n + i] = (float)s2;
        comp *= s / s2;
    }
    opac_out[i] = (float)((double)opac[i] * comp);
}

__global__ __launch_bounds__(kDT) void k_filter_bwd(const float* __restrict__ scales, const float* __restrict__ opac,
                                                    const float* __restrict__ rate, int64_t n, float s_f,
                                                    const float* __restrict__ d_scales_out,
                                                    const float* __restrict__ d_opac_out,
                                                    float* __restrict__ d_scales, float* __restrict__ d_opac) {
    const int64_t i = (int64_t)blockIdx.x * kDT + threadIdx.x;
    if (i >= n) return;
    const double var = filter_var(rate[i], s_f);
    double s[3], s2[3], comp = 1.0;
    for (int k = 0; k < 3; ++k) {
        s[k] = scales[k * n + i];
        s2[k] = sqrt(s[k] * s[k] + var);
        comp *= s[k] / s2[k];
    }
    const double dop = d_opac_out[i];
    const double o2 = (double)opac[i] * comp;
    for (int k = 0; k < 3; ++k) {
        // s' = sqrt(s^2 + var); d log(s / s') / ds = var / (s s'^2)
        const double g = (double)d_scales_out[k * n + i] * s[k] / s2[k] + dop * o2 * var / (s[k] * s2[k] * s2[k]);
        d_scales[k * n + i] = (float)g;
    }
    d_opac[i] = (float)(dop * comp);
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + kDT - 1) / kDT); }

}  // namespace

hipError_t launch_dens_accumulate(const uint32_t* tiles, const float* grad_norm, const float* absgrad,
                                  int32_t n_views, int64_t n, const DensViewScale& sc, float* accum, int32_t* count,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_dens_accumulate, dim3(blocks_of(n)), dim3(kDT), 0, s, tiles, grad_norm,
                       reinterpret_cast<const float2*>(absgrad), n_views, n, sc, accum, count);
    return hipGetLastError();
}

hipError_t launch_dens_classify(const float* accum, const int32_t* count, const float* means, const float* opac,
                                int64_t n, const DensParams& p, uint8_t* action, uint32_t* cand, uint32_t* pruned,
                                uint32_t* key, hipStream_t s) {
    hipLaunchKernelGGL(k_dens_classify, dim3(blocks_of(n)), dim3(kDT), 0, s, accum, count, means, opac, n, p, action,
                       cand, pruned, key);
    return hipGetLastError();
}

hipError_t launch_dens_compact(const uint32_t* cand, const uint32_t* pos, const uint32_t* key, int64_t n,
                               uint32_t* ckey, uint32_t* cidx, hipStream_t s) {
    hipLaunchKernelGGL(k_dens_compact, dim3(blocks_of(n)), dim3(kDT), 0, s, cand, pos, key, n, ckey, cidx);
    return hipGetLastError();
}

hipError_t launch_dens_mark(const uint32_t* sidx, uint32_t k, const uint32_t* cand, bool all, const float* scales,
                            int64_t n, float split_scale, uint8_t* action, hipStream_t s) {
    if (all)
        hipLaunchKernelGGL(k_dens_mark_all, dim3(blocks_of(n)), dim3(kDT), 0, s, cand, scales, n, split_scale,
                           action);
    else if (k)
        hipLaunchKernelGGL(k_dens_mark_sorted, dim3((k + kDT - 1) / kDT), dim3(kDT), 0, s, sidx, k, scales, n,
                           split_scale, action);
    return hipGetLastError();
}

hipError_t launch_filter_rate(const float* means, int64_t n, const ViewTable& vt, bool accumulate, float* rate,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_filter_rate, dim3(blocks_of(n)), dim3(kDT), 0, s, means, n, vt, accumulate ? 1 : 0, rate);
    return hipGetLastError();
}

hipError_t launch_filter_fwd(const float* scales, const float* opac, const float* rate, int64_t n, float s_f,
                             float* scales_out, float* opac_out, hipStream_t s) {
    hipLaunchKernelGGL(k_filter_fwd, dim3(blocks_of(n)), dim3(kDT), 0, s, scales, opac, rate, n, s_f, scales_out,
                       opac_out);
    return hipGetLastError();
}

hipError_t launch_filter_bwd(const float* scales, const float* opac, const float* rate, int64_t n, float s_f,
                             const float* d_scales_out, const float* d_opac_out, float* d_scales, float* d_opac,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_filter_bwd, dim3(blocks_of(n)), dim3(kDT), 0, s, scales, opac, rate, n, s_f, d_scales_out,
                       d_opac_out, d_scales, d_opac);
    return hipGetLastError();
}

}  // namespace gs
