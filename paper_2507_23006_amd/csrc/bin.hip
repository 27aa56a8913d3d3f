// Tile binning -- gfx950.
//
// "Processed in depth order" (§3.1) per tile, ties by input order, is built
// depth-first: slots are sorted once by their 32-bit depth key (N items),
// expanded into (tile, slot) pairs in that order, and the pairs are then
// stably sorted by tile id only (ceil(log2 tiles) bits, 2-3 passes) instead
// of sorting P pairs on a 45-49 bit (tile, depth) key.  Stability of the
// tile sort keeps the depth order inside every tile.
#include "gs_internal.h"

namespace gs {

namespace {

__global__ void k_bin_prepare(const uint32_t* __restrict__ dkey, uint32_t n, uint32_t* __restrict__ keys,
                              uint32_t* __restrict__ slots) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        keys[i] = dkey[i];
        slots[i] = i;
    }
}

// per depth rank: tiles covered and the emission descriptor of its slot
__global__ void k_gather_sorted(const uint32_t* __restrict__ sorted_slot, const uint32_t* __restrict__ tiles,
                                const uint2* __restrict__ rect, uint32_t n, uint32_t* __restrict__ tiles_s,
                                uint2* __restrict__ rect_s) {
    const uint32_t d = blockIdx.x * 256 + threadIdx.x;
    if (d >= n) return;
    const uint32_t s = sorted_slot[d];
    const uint32_t t = tiles[s];
    tiles_s[d] = t;
    rect_s[d] = t ? rect[s] : make_uint2(0u, 1u);
}

constexpr int kEmitThreads = 256;
constexpr int kEmitPer = 4;
constexpr int kEmitChunk = kEmitThreads * kEmitPer;   // pairs per workgroup

// Pair p belongs to the last depth rank d with offsets[d] <= p.  A workgroup
// owns kEmitChunk consecutive pairs, whose ranks form one contiguous run of
// at most kEmitChunk + 1 entries (every visible rank owns >= 1 pair, culled
// ranks own none and sort last); the run's offsets are staged in LDS and
// each pair binary-searches there.  Writes are fully coalesced.
__global__ __launch_bounds__(kEmitThreads) void k_emit_pairs(const uint32_t* __restrict__ offsets,
                                                             const uint2* __restrict__ rect_s,
                                                             const uint32_t* __restrict__ sorted_slot, uint32_t n,
                                                             uint32_t n_pairs, uint32_t* __restrict__ pair_key,
                                                             uint32_t* __restrict__ pair_val) {
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_d0;
    const uint32_t p0 = blockIdx.x * kEmitChunk;
    if (threadIdx.x == 0) {
        // last d with offsets[d] <= p0 (offsets[0] == 0 <= p0)
        uint32_t lo = 0, hi = n;      // invariant: offsets[lo] <= p0, answer in [lo, hi)
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (offsets[mid] <= p0) lo = mid; else hi = mid;
        }
        s_d0 = lo;
    }
    __syncthreads();
    const uint32_t d0 = s_d0;
    const uint32_t cnt = min((uint32_t)(kEmitChunk + 1), n - d0);
    for (uint32_t i = threadIdx.x; i < kEmitChunk + 1; i += kEmitThreads)
        s_off[i] = i < cnt ? offsets[d0 + i] : 0xFFFFFFFFu;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) {
        const uint32_t p = p0 + k * kEmitThreads + threadIdx.x;
        if (p >= n_pairs) break;
        uint32_t lo = 0, hi = cnt;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= p) lo = mid; else hi = mid;
        }
        const uint32_t d = d0 + lo;
        const uint32_t local = p - s_off[lo];
        const uint2 rs = rect_s[d];
        const uint32_t w = rs.y & 0xFFFFu, tw = rs.y >> 16;
        const uint32_t row = local / w, col = local - row * w;
        pair_key[p] = rs.x + row * tw + col;
        pair_val[p] = sorted_slot[d];
    }
}

__global__ void k_tile_ranges(const uint32_t* __restrict__ keys, uint32_t n, uint2* __restrict__ ranges,
                              uint32_t n_tiles) {
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const uint32_t k = keys[p];
    if (k >= n_tiles) return;     // keys are tile ids by construction; guards the write
    if (p == 0 || keys[p - 1] != k) ranges[k].x = p;
    if (p == n - 1 || keys[p + 1] != k) ranges[k].y = p + 1;
}

}  // namespace

hipError_t launch_bin_prepare(const Projected& proj, uint32_t n_slots, uint32_t* keys, uint32_t* slots,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_bin_prepare, dim3((n_slots + 255) / 256), dim3(256), 0, s, proj.dkey, n_slots, keys, slots);
    return hipGetLastError();
}

hipError_t launch_gather_sorted(const uint32_t* sorted_slot, const Projected& proj, uint32_t n_slots,
                                uint32_t* tiles_s, uint2* rect_s, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_sorted, dim3((n_slots + 255) / 256), dim3(256), 0, s, sorted_slot, proj.tiles,
                       proj.rect, n_slots, tiles_s, rect_s);
    return hipGetLastError();
}

hipError_t launch_emit_pairs(const uint32_t* offsets, const uint2* rect_s, const uint32_t* sorted_slot,
                             uint32_t n_slots, uint32_t n_pairs, uint32_t* pair_key, uint32_t* pair_val,
                             hipStream_t s) {
    if (!n_pairs) return hipSuccess;
    const uint32_t blocks = (n_pairs + kEmitChunk - 1) / kEmitChunk;
    hipLaunchKernelGGL(k_emit_pairs, dim3(blocks), dim3(kEmitThreads), 0, s, offsets, rect_s, sorted_slot, n_slots,
                       n_pairs, pair_key, pair_val);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* sorted_keys, uint32_t n_pairs, uint32_t* ranges, uint32_t n_tiles,
                              hipStream_t s) {
    hipError_t e = fill_u32(ranges, 0u, (size_t)n_tiles * 2, s);
    if (e != hipSuccess || !n_pairs) return e;
    hipLaunchKernelGGL(k_tile_ranges, dim3((n_pairs + 255) / 256), dim3(256), 0, s, sorted_keys, n_pairs,
                       reinterpret_cast<uint2*>(ranges), n_tiles);
    return hipGetLastError();
}

}  // namespace gs
