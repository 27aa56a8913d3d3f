// Front-to-back compositing (Eq. 2) and its backward -- gfx950.
//
// One 256-thread workgroup (four wave64s) per 16x16 tile, one pixel per
// thread.  The tile's depth-ordered list is walked in batches: each thread
// gathers one projected record (three 16-byte loads) into LDS, then every
// thread evaluates the whole batch from LDS; all lanes of a wave read the
// same record, which the LDS serves as a conflict-free broadcast.  The
// forward keeps no per-pixel lists: it stores the final transmittance and
// the position of the last composited entry, and the backward walks the
// list back to front, recovering T_i = T_{i+1} / (1 - alpha_i).
//
// Backward per entry: gradients are summed over the wave with DPP
// row-shift / row-broadcast adds (six VALU steps, result in lane 63),
// across the four waves in LDS, and then added to the per-slot 2D gradient
// buffer with one float atomic per nonzero field.
#include "gs_internal.h"

namespace gs {

namespace {

// alpha of record (a, b) at pixel centre (px, py): the same instruction
// sequence in forward and backward, so skip and stop decisions agree bit
// for bit.
struct Eval {
    float dx, dy, G, raw, alpha;
    bool keep;   // not skipped (power <= 0 and alpha >= 1/255)
};

__device__ __forceinline__ Eval eval_entry(const float4 a, const float4 b, float px, float py) {
    Eval e;
    e.dx = px - a.x;
    e.dy = py - a.y;
    const float p2 = fmaf(a.z, e.dx * e.dx, fmaf(a.w, e.dx * e.dy, b.x * (e.dy * e.dy)));
    e.G = __builtin_amdgcn_exp2f(p2);
    e.raw = b.y * e.G;
    e.alpha = fminf(kAlphaMax, e.raw);
    e.keep = !(p2 > 0.0f) && e.alpha >= kAlphaMin;
    return e;
}

// Record -> LDS form: the mean relative to the tile origin (integer part
// minus the origin is exact; adding the stored fraction rounds once, at the
// scale of the tile rather than of the image).
__device__ __forceinline__ float4 stage_geom(const float4 r0, const float4 r1, const float4 r2, float ox, float oy) {
    return make_float4((r0.x - ox) + r1.w, (r0.y - oy) + r2.w, r0.z, r0.w);
}

constexpr int kFwdBatch = 256;

__global__ __launch_bounds__(256) void k_render_fwd(const float4* __restrict__ rec,
                                                    const uint32_t* __restrict__ pair_vals,
                                                    const uint2* __restrict__ ranges, ViewTable vt, OptK opt,
                                                    float* __restrict__ rgb, float* __restrict__ depth,
                                                    float* __restrict__ alpha_out, float* __restrict__ T_out,
                                                    int32_t* __restrict__ last_out) {
    __shared__ float4 s0[kFwdBatch], s1[kFwdBatch], s2[kFwdBatch];
    const int tile = blockIdx.x;
    const int v = view_of_tile(vt, tile);
    const ViewK& V = vt.v[v];
    const int lt = tile - V.tile_off;
    const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
    const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
    const bool inside = px < V.W && py < V.H;
    const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
    const float fpx = (float)(threadIdx.x & 15) + 0.5f, fpy = (float)(threadIdx.x >> 4) + 0.5f;
    const uint2 rg = ranges[tile];

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, D = 0.0f;
    int last = 0;
    bool done = !inside;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kFwdBatch) {
        // barrier: every pixel of the tile done ends the walk; also guards LDS reuse
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t j = b0 + threadIdx.x;
        if (j < rg.y) {
            const uint32_t s = pair_vals[j];
            const float4 r0 = rec[3 * (size_t)s + 0], r1 = rec[3 * (size_t)s + 1], r2 = rec[3 * (size_t)s + 2];
            s0[threadIdx.x] = stage_geom(r0, r1, r2, ox, oy);
            s1[threadIdx.x] = r1;
            s2[threadIdx.x] = r2;
        }
        __syncthreads();
        if (!done) {
            const int cnt = (int)min((uint32_t)kFwdBatch, rg.y - b0);
            for (int k = 0; k < cnt; ++k) {
                const float4 a = s0[k], b = s1[k];
                const Eval e = eval_entry(a, b, fpx, fpy);
                if (!e.keep) continue;
                const float Tn = T * (1.0f - e.alpha);
                if (Tn < kTMin) {
                    done = true;
                    break;
                }
                const float4 c = s2[k];
                const float w = e.alpha * T;
                c0 = fmaf(c.x, w, c0);
                c1 = fmaf(c.y, w, c1);
                c2 = fmaf(c.z, w, c2);
                D = fmaf(b.z, w, D);
                T = Tn;
                last = (int)(b0 - rg.x) + k + 1;
            }
        }
    }
    if (!inside) return;
    const int64_t pix = V.pix_off + (int64_t)py * V.W + px;
    rgb[3 * pix + 0] = fmaf(T, opt.bg[0], c0);
    rgb[3 * pix + 1] = fmaf(T, opt.bg[1], c1);
    rgb[3 * pix + 2] = fmaf(T, opt.bg[2], c2);
    depth[pix] = D;
    alpha_out[pix] = 1.0f - T;
    T_out[pix] = T;
    last_out[pix] = last;
}

// Per pixel: how many list entries the forward must evaluate (up to and
// including the one that stops the pixel, else the whole list).  The unit
// of work of compositing; used for the roofline, never on the render path.
__global__ __launch_bounds__(256) void k_render_count(const float4* __restrict__ rec,
                                                      const uint32_t* __restrict__ pair_vals,
                                                      const uint2* __restrict__ ranges, ViewTable vt,
                                                      int32_t* __restrict__ n_eval) {
    __shared__ float4 s0[kFwdBatch], s1[kFwdBatch];
    const int tile = blockIdx.x;
    const int v = view_of_tile(vt, tile);
    const ViewK& V = vt.v[v];
    const int lt = tile - V.tile_off;
    const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
    const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
    const bool inside = px < V.W && py < V.H;
    const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
    const float fpx = (float)(threadIdx.x & 15) + 0.5f, fpy = (float)(threadIdx.x >> 4) + 0.5f;
    const uint2 rg = ranges[tile];
    float T = 1.0f;
    int count = 0;
    bool done = !inside;
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kFwdBatch) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t j = b0 + threadIdx.x;
        if (j < rg.y) {
            const uint32_t s = pair_vals[j];
            const float4 r0 = rec[3 * (size_t)s + 0], r1 = rec[3 * (size_t)s + 1], r2 = rec[3 * (size_t)s + 2];
            s0[threadIdx.x] = stage_geom(r0, r1, r2, ox, oy);
            s1[threadIdx.x] = r1;
        }
        __syncthreads();
        if (!done) {
            const int cnt = (int)min((uint32_t)kFwdBatch, rg.y - b0);
            for (int k = 0; k < cnt; ++k) {
                ++count;
                const Eval e = eval_entry(s0[k], s1[k], fpx, fpy);
                if (!e.keep) continue;
                const float Tn = T * (1.0f - e.alpha);
                if (Tn < kTMin) {
                    done = true;
                    break;
                }
                T = Tn;
            }
        }
    }
    if (inside) n_eval[V.pix_off + (int64_t)py * V.W + px] = count;
}

// sum over the 64 lanes; lane 63 holds the result
__device__ __forceinline__ float wave_sum_lane63(float x) {
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

constexpr int kBwdBatch = 64;
constexpr int kG2 = 12;   // per-slot 2D gradient fields

__global__ __launch_bounds__(256) void k_render_bwd(const float4* __restrict__ rec,
                                                    const uint32_t* __restrict__ pair_vals,
                                                    const uint2* __restrict__ ranges, ViewTable vt, OptK opt,
                                                    const float* __restrict__ T_final,
                                                    const int32_t* __restrict__ last_in,
                                                    const float* __restrict__ d_rgb, const float* __restrict__ d_depth,
                                                    const float* __restrict__ d_alpha, float* __restrict__ grad2d) {
    __shared__ float4 s0[kBwdBatch], s1[kBwdBatch], s2[kBwdBatch];
    __shared__ uint32_t s_slot[kBwdBatch];
    __shared__ float s_red[4][kBwdBatch][kG2];
    __shared__ int s_maxlast;

    const int tile = blockIdx.x;
    const int v = view_of_tile(vt, tile);
    const ViewK& V = vt.v[v];
    const int lt = tile - V.tile_off;
    const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
    const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
    const bool inside = px < V.W && py < V.H;
    const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
    const float fpx = (float)(threadIdx.x & 15) + 0.5f, fpy = (float)(threadIdx.x >> 4) + 0.5f;
    const uint2 rg = ranges[tile];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    float T = 1.0f, gC0 = 0.0f, gC1 = 0.0f, gC2 = 0.0f, gD = 0.0f, gA = 0.0f;
    int last = 0;
    if (inside) {
        const int64_t pix = V.pix_off + (int64_t)py * V.W + px;
        T = T_final[pix];
        last = last_in[pix];
        if (d_rgb) {
            gC0 = d_rgb[3 * pix + 0];
            gC1 = d_rgb[3 * pix + 1];
            gC2 = d_rgb[3 * pix + 2];
        }
        if (d_depth) gD = d_depth[pix];
        if (d_alpha) gA = d_alpha[pix];
    }
    if (threadIdx.x == 0) s_maxlast = 0;
    __syncthreads();
    if (last > 0) atomicMax(&s_maxlast, last);
    __syncthreads();
    const int maxlast = s_maxlast;

    // R = remaining colour behind the entry divided by T after it; starts at bg
    float R0 = opt.bg[0], R1 = opt.bg[1], R2 = opt.bg[2], RD = 0.0f, Q = 1.0f;
    const float ln2 = kLn2;

    for (int b_end = maxlast; b_end > 0; b_end -= kBwdBatch) {
        const int b_start = max(0, b_end - kBwdBatch);
        const int cnt = b_end - b_start;
        __syncthreads();   // previous batch fully consumed
        if ((int)threadIdx.x < cnt) {
            const uint32_t s = pair_vals[rg.x + b_start + threadIdx.x];
            s_slot[threadIdx.x] = s;
            const float4 r0 = rec[3 * (size_t)s + 0], r1 = rec[3 * (size_t)s + 1], r2 = rec[3 * (size_t)s + 2];
            s0[threadIdx.x] = stage_geom(r0, r1, r2, ox, oy);
            s1[threadIdx.x] = r1;
            s2[threadIdx.x] = r2;
        }
        __syncthreads();
        for (int k = cnt - 1; k >= 0; --k) {
            const int pos = b_start + k;           // 0-based position in the tile list
            const float4 a = s0[k], b = s1[k], c = s2[k];
            const Eval e = eval_entry(a, b, fpx, fpy);
            const bool contrib = pos < last && e.keep;
            float g[kG2];
#pragma unroll
            for (int f = 0; f < kG2; ++f) g[f] = 0.0f;
            if (contrib) {
                const float one_m = 1.0f - e.alpha;
                const float Ti = T * __builtin_amdgcn_rcpf(one_m);
                const float w = e.alpha * Ti;
                const float dal = Ti * (gC0 * (c.x - R0) + gC1 * (c.y - R1) + gC2 * (c.z - R2) + gD * (b.z - RD) +
                                        gA * Q);
                g[6] = gC0 * w;
                g[7] = gC1 * w;
                g[8] = gC2 * w;
                g[9] = gD * w;
                if (e.raw < kAlphaMax) {
                    g[5] = dal * e.G;
                    const float dp = dal * e.alpha;          // dL/d power
                    // conic (A, B, C) = -ln2 (2 qa, qb, 2 qc)
                    const float dmx = -dp * ln2 * (2.0f * a.z * e.dx + a.w * e.dy);
                    const float dmy = -dp * ln2 * (a.w * e.dx + 2.0f * b.x * e.dy);
                    g[0] = dmx;
                    g[1] = dmy;
                    g[2] = -0.5f * e.dx * e.dx * dp;
                    g[3] = -e.dx * e.dy * dp;
                    g[4] = -0.5f * e.dy * e.dy * dp;
                    g[10] = fabsf(dmx);
                    g[11] = fabsf(dmy);
                }
                R0 = fmaf(R0, one_m, c.x * e.alpha);
                R1 = fmaf(R1, one_m, c.y * e.alpha);
                R2 = fmaf(R2, one_m, c.z * e.alpha);
                RD = fmaf(RD, one_m, b.z * e.alpha);
                Q *= one_m;
                T = Ti;
            }
            if (__ballot(contrib)) {
#pragma unroll
                for (int f = 0; f < kG2; ++f) g[f] = wave_sum_lane63(g[f]);
                if (lane == 63) {
#pragma unroll
                    for (int f = 0; f < kG2; ++f) s_red[wave][k][f] = g[f];
                }
            } else if (lane == 0) {
#pragma unroll
                for (int f = 0; f < kG2; ++f) s_red[wave][k][f] = 0.0f;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * kG2; i += 256) {
            const int k = i / kG2, f = i - k * kG2;
            const float sum = s_red[0][k][f] + s_red[1][k][f] + s_red[2][k][f] + s_red[3][k][f];
            if (sum != 0.0f) atomicAdd(&grad2d[(size_t)s_slot[k] * kG2 + f], sum);
        }
    }
}

}  // namespace

hipError_t launch_render_fwd(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                             const ViewTable& vt, const OptK& opt, float* rgb, float* depth, float* alpha,
                             float* T_final, int32_t* last, hipStream_t s) {
    if (vt.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_render_fwd, dim3(vt.total_tiles), dim3(256), 0, s, proj.rec, pair_vals, ranges, vt, opt, rgb,
                       depth, alpha, T_final, last);
    return hipGetLastError();
}

hipError_t launch_render_count(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                               const ViewTable& vt, int32_t* n_eval, hipStream_t s) {
    if (vt.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_render_count, dim3(vt.total_tiles), dim3(256), 0, s, proj.rec, pair_vals, ranges, vt, n_eval);
    return hipGetLastError();
}

hipError_t launch_render_bwd(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                             const ViewTable& vt, const OptK& opt, const float* T_final, const int32_t* last,
                             const float* d_rgb, const float* d_depth, const float* d_alpha, float* grad2d,
                             hipStream_t s) {
    if (vt.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_render_bwd, dim3(vt.total_tiles), dim3(256), 0, s, proj.rec, pair_vals, ranges, vt, opt,
                       T_final, last, d_rgb, d_depth, d_alpha, grad2d);
    return hipGetLastError();
}

}  // namespace gs
