// Internal definitions shared by the gfx950 kernels and the host side of
// the library.  Not part of the public ABI (include/gs.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gs {

constexpr int kTile = GS_TILE;
constexpr int kTilePix = kTile * kTile;       // 256 pixels = 4 wave64s
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr double kLog2e = 1.4426950408889634;
constexpr float kLn2 = 0.6931471805599453f;

// Per-view constants, passed by value in kernel arguments (the whole table
// stays under 3 KB).  Camera inputs are float32, so they are kept as float
// and widened exactly in the kernels; quantities derived on the host are
// double because projection runs in FP64 (it is HBM-bound, and FP64 VALU on
// CDNA4 peaks as high as non-packed FP32).
struct ViewK {
    float R[9];           // world -> camera rotation, row-major
    float t[3];
    float fx, fy, cx, cy;
    float znear, zfar;
    double campos[3];     // camera centre in world space, -R^T t
    double ulo, uhi, vlo, vhi;   // Jacobian clamp of x/z and y/z
    int32_t W, H, tiles_x, tiles_y;
    int32_t tile_off;     // first global tile id of this view
    int32_t pad;
    int64_t pix_off;      // first global pixel of this view
};

struct ViewTable {
    ViewK v[GS_MAX_VIEWS];
    int32_t n_views;
    int32_t total_tiles;
};

struct OptK {
    int32_t sh_degree;
    float dilation;
    int32_t aa;
    float bg[3];
};

// Map a global tile id to its view (views are few; linear scan of kernargs).
__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int tile) {
    int v = 0;
    for (int i = 1; i < vt.n_views; ++i)
        if (tile >= vt.v[i].tile_off) v = i;
    return v;
}

// Real SH with the Condon-Shortley phase (m = -l..l per band), degree <= 3,
// as polynomials valid on the unit sphere.  The constants are the
// normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times sqrt(2) for
// m != 0, reduced to closed forms:
//   k0 = 1/(2 sqrt(pi)), k1 = sqrt(3/(4 pi)), k2 = sqrt(15/pi)/2,
//   k6 = sqrt(5/pi)/4, k8 = sqrt(15/pi)/4, k9 = sqrt(35/(2 pi))/4,
//   k10 = sqrt(105/pi)/2, k11 = sqrt(21/(2 pi))/4, k12 = sqrt(7/pi)/4,
//   k14 = sqrt(105/pi)/4.
struct ShK {
    static constexpr double k0 = 0.28209479177387814;
    static constexpr double k1 = 0.4886025119029199;
    static constexpr double k2 = 1.0925484305920792;
    static constexpr double k6 = 0.31539156525252005;
    static constexpr double k8 = 0.5462742152960396;
    static constexpr double k9 = 0.5900435899266435;
    static constexpr double k10 = 2.890611442640554;
    static constexpr double k11 = 0.4570457994644658;
    static constexpr double k12 = 0.3731763325901154;
    static constexpr double k14 = 1.445305721320277;
};

template <class Real>
__device__ __forceinline__ void sh_eval_basis(Real x, Real y, Real z, int degree, Real Y[16]) {
    Y[0] = (Real)ShK::k0;
    if (degree < 1) return;
    Y[1] = -(Real)ShK::k1 * y;
    Y[2] = (Real)ShK::k1 * z;
    Y[3] = -(Real)ShK::k1 * x;
    if (degree < 2) return;
    const Real xx = x * x, yy = y * y, zz = z * z;
    Y[4] = (Real)ShK::k2 * x * y;
    Y[5] = -(Real)ShK::k2 * y * z;
    Y[6] = (Real)ShK::k6 * ((Real)2 * zz - xx - yy);
    Y[7] = -(Real)ShK::k2 * x * z;
    Y[8] = (Real)ShK::k8 * (xx - yy);
    if (degree < 3) return;
    Y[9] = -(Real)ShK::k9 * y * ((Real)3 * xx - yy);
    Y[10] = (Real)ShK::k10 * x * y * z;
    Y[11] = -(Real)ShK::k11 * y * ((Real)4 * zz - xx - yy);
    Y[12] = (Real)ShK::k12 * z * ((Real)2 * zz - (Real)3 * xx - (Real)3 * yy);
    Y[13] = -(Real)ShK::k11 * x * ((Real)4 * zz - xx - yy);
    Y[14] = (Real)ShK::k14 * z * (xx - yy);
    Y[15] = -(Real)ShK::k9 * x * (xx - (Real)3 * yy);
}

// In-place exclusive scan of 256 counters in LDS by one whole wave (the
// calling threads are exactly the 64 lanes of one wave), four per lane.
__device__ __forceinline__ void wave_excl_scan256(uint32_t* c) {
    const uint32_t l = threadIdx.x & 63u;
    const uint32_t a0 = c[4 * l], a1 = c[4 * l + 1], a2 = c[4 * l + 2], a3 = c[4 * l + 3];
    const uint32_t sum = a0 + a1 + a2 + a3;
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if ((int)l >= off) incl += y;
    }
    const uint32_t base = incl - sum;
    c[4 * l] = base;
    c[4 * l + 1] = base + a0;
    c[4 * l + 2] = base + a0 + a1;
    c[4 * l + 3] = base + a0 + a1 + a2;
}

// Copies the first cnt entries of a workgroup's list (local index | view
// mask << 16) to out, grouped by the mask's low 8 bits, so that the lanes
// of a wave share few views and a loop over the views of a launch runs
// fewer passes per wave.  The order inside a group is arbitrary (each entry
// is handled alone, so results do not depend on it).  Every thread of the
// workgroup (at least 64) calls it; hist holds 256 counters.
__device__ __forceinline__ void group_by_views(const uint32_t* list, uint32_t cnt, uint32_t* out, uint32_t* hist) {
    for (uint32_t b = threadIdx.x; b < 256u; b += blockDim.x) hist[b] = 0u;
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) atomicAdd(&hist[(list[j] >> 16) & 255u], 1u);
    __syncthreads();
    if (threadIdx.x < 64) wave_excl_scan256(hist);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += blockDim.x) {
        const uint32_t e = list[j];
        out[atomicAdd(&hist[(e >> 16) & 255u], 1u)] = e;
    }
    __syncthreads();
}

}  // namespace gs

// ---------------------------------------------------------------------------
// host-side launch helpers (defined in the .hip sources)
// ---------------------------------------------------------------------------
namespace gs {

// ---------------------------------------------------------------------------
// measurement: while enabled (gs_kernel_timing), the launch helpers of the
// timed kernels bracket their launch with two events on the launch stream;
// timer_begin returns the closing event (null when disabled)
// ---------------------------------------------------------------------------
hipEvent_t timer_begin(int kernel, hipStream_t s);
void timer_end(hipEvent_t closing, hipStream_t s);


struct Projected {
    float4* rec;          // [slots][4]
    uint2* rect;          // [slots]
    uint32_t* tiles;      // [slots]
    uint32_t* dkey;       // [slots]
    uint32_t* tile_order; // [tiles] compositing launch order, or null for tile index order
    uint64_t* tile_mask;  // [slots] covered tiles of rectangles of <= 64 tiles (0: all), or null
};

// app: appearance offsets [n][4] (dc, do) or null
struct GaussPtrs {
    const float *means, *scales, *quats, *opac, *sh;
    const float *app;
};

struct GradPtrs {
    float *means, *scales, *quats, *opac, *sh;
    float *app;
};

hipError_t launch_project_fwd(const GaussPtrs& g, int64_t n, const ViewTable& vt, const OptK& opt,
                              const Projected& out, hipStream_t s);

// a run of consecutive Gaussians [gstart, gstart + len) projected into view
// `view` at slots [slot_start, slot_start + len); len is implied by the next
// segment's slot_start (or the slot count)
struct SlotSeg {
    int64_t gstart;
    uint32_t slot_start;
    uint32_t view;
};

hipError_t launch_project_slots(const GaussPtrs& g, int64_t n, const ViewTable& vt, const OptK& opt,
                                const SlotSeg* segs, int32_t n_seg, uint32_t n_slots, const Projected& out,
                                hipStream_t s);

// radix sort / scan primitives (sort.hip)
// n_dev (nullable): the element count on the device, at most n, which sizes
// the launches (no host read-back needed)
size_t radix_hist_elems(uint32_t n);        // counters needed per pass
int radix_passes(uint32_t n, int begin_bit, int end_bit);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                            uint32_t n, int begin_bit, int end_bit, uint32_t* hist, hipStream_t s,
                            bool* result_in_alt, const uint32_t* n_dev = nullptr, bool small_tiles = false);
size_t scan_tmp_elems(uint32_t n);
// with n_dev, the scanned count is ceil(*n_dev / div) * mul, at most n
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tmp,
                              unsigned long long* total, hipStream_t s, const uint32_t* n_dev = nullptr,
                              uint32_t div = 1, uint32_t mul = 1);
// exclusive scan of (in[i] != 0); the sum of in[] itself is added to
// sum_parts (kBinPairParts partial sums, 16 u64 apart, zeroed by the caller)
hipError_t exclusive_scan_nonzero_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tmp,
                                      unsigned long long* total, unsigned long long* sum_parts, hipStream_t s);
hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
// zero the [12]-float 2D-gradient rows of slots with tiles > 0
hipError_t zero_seen_grad2d(const uint32_t* tiles, float* grad2d, int64_t n_slots, hipStream_t s);

// binning (bin.hip)
// pair counts are summed into kBinPairParts partial sums, 16 u64 apart
constexpr int kBinPairParts = 64;
// compaction of the visible slots: depth keys, their positions as sort
// values, and per position a 32-byte descriptor (uint4 pair: rect.x, rect.y,
// mask lo, mask hi; tiles, slot, 0, 0)
hipError_t launch_compact_visible(const Projected& proj, const uint32_t* pos, uint32_t n_slots, uint32_t* keys,
                                  uint32_t* vals, uint4* desc, hipStream_t s);
hipError_t launch_gather_sorted(const uint32_t* sorted_pos, const uint4* desc, uint32_t n_visible, const uint32_t* counts,
                                uint32_t* tiles_s, uint2* rect_s, uint64_t* mask_s, uint32_t* slot_s, hipStream_t s);
// gather, emission and ranges take their counts from the device (counts[0]
// visible ranks, counts[1] pairs, from launch_bin_counts) when counts is
// set, within the launch bounds n_visible / n_slots, n_pairs
hipError_t launch_emit_pairs(const uint32_t* offsets, const uint2* rect_s, const uint64_t* mask_s,
                             const uint32_t* sorted_slot, uint32_t n_slots, uint32_t n_pairs, const uint32_t* counts,
                             uint32_t* pair_key, uint32_t* pair_val, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t* sorted_keys, uint32_t n_pairs, const uint32_t* counts, uint32_t* ranges,
                              uint32_t n_tiles, hipStream_t s);
// total[0] = visible slots, parts = kBinPairParts pair-count parts (16
// apart): writes the pair count to n_pairs_out and the effective counts
// counts[0..1], 0 when the pairs exceed capacity
hipError_t launch_bin_counts(const unsigned long long* total, const unsigned long long* parts,
                             unsigned long long capacity, int64_t* n_pairs_out, uint32_t* counts, hipStream_t s);
// tile launch order for compositing, longest lists first
hipError_t launch_tile_order(const uint32_t* ranges, uint32_t n_tiles, uint32_t* order, hipStream_t s);

// Segmented compositing: lists longer than kSegLen positions are walked in
// segments of kSegLen by separate workgroups, forward and backward.
// work_off [T + 1] and state_off [T + 1] are exclusive prefix sums, over the
// tiles in launch order, of the work items (segments) and of the stored
// segment states (segments 1 .. n - 1 of a segmented tile); state holds
// kSegFields planes of 256 pixels per stored segment: T_seg, C_seg (r, g,
// b), D_seg and (int) the position of the segment's last entry; stop_seg
// [T][256] (by tile) is the segment a pixel stops in, -1 for none, for the
// segmented forward.
constexpr int kSegLen = 512;
constexpr int kSegFields = 6;
struct SegPlan {
    uint32_t* work_off;    // null: one work item per tile, no segments
    uint32_t* state_off;
    float* state;
    uint32_t n_tiles;
    int32_t* stop_seg;
    uint32_t capacity;     // stored states the area holds
};
// plans the segments of every tile (segments disabled when they need more
// than `capacity` stored states)
hipError_t launch_seg_plan(const Projected& proj, const uint2* ranges, const ViewTable& vt, uint32_t capacity,
                           const SegPlan& plan, hipStream_t s);
// the plan, then the states by a walk of the stored segments
hipError_t launch_seg_prepare(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                              const ViewTable& vt, const int32_t* last, uint32_t capacity, const SegPlan& plan,
                              hipStream_t s);

// compositing (render.hip)
// persistent_ctas > 0: a grid of that many workgroups pulling tiles from
// `work` (one u32, zeroed here by a fill kernel); plan (one workgroup per
// tile only): also write the segment states of the planned tiles
hipError_t launch_render_fwd(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                             const ViewTable& vt, const OptK& opt, float* rgb, float* depth, float* alpha,
                             float* T_final, int32_t* last, hipStream_t s,
                             int persistent_ctas = 0, uint32_t* work = nullptr, const SegPlan* plan = nullptr);
hipError_t launch_render_count(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                               const ViewTable& vt, int32_t* n_eval, hipStream_t s);
hipError_t launch_render_bwd(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                             const ViewTable& vt, const OptK& opt, const float* T_final, const int32_t* last,
                             const float* d_rgb, const float* d_depth, const float* d_alpha, float* grad2d,
                             const SegPlan& plan, uint32_t capacity, bool abs_sums, hipStream_t s);

// training loss (loss.hip): per-workgroup partial sums, then a fixed-order total
size_t loss_partials(int64_t n_pix);
// the allocation-free loss: largest pixel count its file-scope scratch
// holds, and that scratch's address on the current device
int64_t loss_scratch_max_pixels();
hipError_t loss_scratch_ptr(double** out);
hipError_t launch_loss(const float* rgb, const float* depth, const float* alpha, const float* t_rgb,
                       const float* t_depth, int64_t n_pix, float lambda, float* loss, float* d_rgb, float* d_depth,
                       float* d_alpha, double* partial, hipStream_t s);

// D-SSIM term (ssim.hip)
size_t ssim_partials(int W, int H);
hipError_t launch_dssim(const float* x, const float* y, int W, int H, float weight, float* loss, float* dx, float* Pa,
                        float* Pb, float* Pc, double* partial, hipStream_t s);

// projection backward (project_bwd.hip)
// grads_zeroed: the outputs hold zeros already (launch_zero_grads); only the
// rows of Gaussians some view sees are written
hipError_t launch_project_bwd(const GaussPtrs& g, int64_t n, const ViewTable& vt, const OptK& opt,
                              const Projected& proj, const float* grad2d, const GradPtrs& out,
                              float* mean2d_norm, float* absgrad, hipStream_t s, bool grads_zeroed = false);
// zeroes every parameter-gradient array of n Gaussians (narrow grid)
hipError_t launch_zero_grads(const GradPtrs& out, int64_t n, hipStream_t s);

// appearance transform MLP (appearance.hip)
struct AppMlp {
    const float *w1, *b1, *w2, *b2;
};
struct AppGrad {
    float *d_w1, *d_b1, *d_w2, *d_b2, *d_iemb;
};
size_t app_workspace_bytes(int64_t n);

// densification bookkeeping and the 3D filter (densify.hip)
struct DensViewScale {
    float s[GS_MAX_VIEWS];
};
struct DensParams {
    double box_min[3], box_max[3];
    float tau_min, eta, d_max, prune_opacity;
};
hipError_t launch_dens_accumulate(const uint32_t* tiles, const float* grad_norm, const float* absgrad,
                                  int32_t n_views, int64_t n, const DensViewScale& sc, float* accum, int32_t* count,
                                  hipStream_t s);
hipError_t launch_dens_classify(const float* accum, const int32_t* count, const float* means, const float* opac,
                                int64_t n, const DensParams& p, uint8_t* action, uint32_t* cand, uint32_t* pruned,
                                uint32_t* key, hipStream_t s);
hipError_t launch_dens_compact(const uint32_t* cand, const uint32_t* pos, const uint32_t* key, int64_t n,
                               uint32_t* ckey, uint32_t* cidx, hipStream_t s);
hipError_t launch_dens_mark(const uint32_t* sidx, uint32_t k, const uint32_t* cand, bool all, const float* scales,
                            int64_t n, float split_scale, uint8_t* action, hipStream_t s);
hipError_t launch_filter_rate(const float* means, int64_t n, const ViewTable& vt, bool accumulate, float* rate,
                              hipStream_t s);
hipError_t launch_filter_fwd(const float* scales, const float* opac, const float* rate, int64_t n, float s_f,
                             float* scales_out, float* opac_out, hipStream_t s);
hipError_t launch_filter_bwd(const float* scales, const float* opac, const float* rate, int64_t n, float s_f,
                             const float* d_scales_out, const float* d_opac_out, float* d_scales, float* d_opac,
                             hipStream_t s);
hipError_t launch_app_fwd(const float* gemb, int64_t n, const float* iemb, const AppMlp& w, float reg_weight,
                          float* offsets, float* reg_value, void* ws, hipStream_t s);
hipError_t launch_app_bwd(const float* gemb, int64_t n, const float* iemb, const AppMlp& w, const float* offsets,
                          const float* d_offsets, const float* d_reg, float reg_weight, float* d_gemb,
                          const AppGrad& g, void* ws, hipStream_t s);

}  // namespace gs
