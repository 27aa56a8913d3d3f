// Tile binning -- gfx950.
//
// "Processed in depth order" (§3.1) per tile, ties by input order, is built
// depth-first: the visible slots are compacted in slot order (a scan), sorted
// once by their 32-bit depth key, expanded into (tile, slot) pairs in that
// order, and the pairs are then stably sorted by tile id only
// (ceil(log2 tiles) bits, 2-3 passes) instead of sorting P pairs on a 45-49
// bit (tile, depth) key.  Stability of both sorts keeps the depth order
// inside every tile, ties by slot index.
#include "gs_internal.h"

namespace gs {

namespace {

// Visible slots, in slot order, with their depth keys: the input of the
// depth sort (culled slots never enter it), whose values are the compaction
// positions.  Each visible slot also leaves a 32-byte descriptor there
// (rectangle, tile mask, tile count, slot) so that the gather after the sort
// fetches one line per depth rank instead of one per array.
__global__ __launch_bounds__(256) void k_compact_visible(const uint32_t* __restrict__ tiles,
                                                         const uint32_t* __restrict__ pos,
                                                         const uint32_t* __restrict__ dkey,
                                                         const uint2* __restrict__ rect,
                                                         const uint64_t* __restrict__ mask, uint32_t n,
                                                         uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                         uint4* __restrict__ desc) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = tiles[i];
    if (!t) return;
    const uint32_t d = pos[i];
    keys[d] = dkey[i];
    vals[d] = d;
    const uint2 r = rect[i];
    const uint64_t m = mask ? mask[i] : 0ull;
    desc[2 * d] = make_uint4(r.x, r.y, (uint32_t)m, (uint32_t)(m >> 32));
    desc[2 * d + 1] = make_uint4(t, i, 0u, 0u);
}

// per depth rank: tiles covered and the emission descriptor of its slot
// (rectangle, covered-tile mask, slot), from its compaction descriptor
__global__ void k_gather_sorted(const uint32_t* __restrict__ sorted_pos, const uint4* __restrict__ desc,
                                uint32_t n_max, const uint32_t* __restrict__ counts, uint32_t* __restrict__ tiles_s,
                                uint2* __restrict__ rect_s, uint64_t* __restrict__ mask_s,
                                uint32_t* __restrict__ slot_s) {
    const uint32_t n = counts ? min(counts[0], n_max) : n_max;
    const uint32_t d = blockIdx.x * 256 + threadIdx.x;
    if (d >= n) return;
    const uint32_t c = sorted_pos[d];
    const uint4 a = desc[2 * c], b = desc[2 * c + 1];
    tiles_s[d] = b.x;
    rect_s[d] = make_uint2(a.x, a.y);
    mask_s[d] = (uint64_t)a.z | ((uint64_t)a.w << 32);
    slot_s[d] = b.y;
}

// index of the k-th set bit (k < popcount(m)) of m, by halving
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t k) {
    uint32_t base = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const uint64_t low = m & ((1ull << width) - 1ull);
        const uint32_t c = (uint32_t)__popcll(low);
        if (k >= c) {
            k -= c;
            m >>= width;
            base += width;
        } else {
            m = low;
        }
    }
    return base;
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
                                                             const uint64_t* __restrict__ mask_s,
                                                             const uint32_t* __restrict__ sorted_slot, uint32_t n_max,
                                                             uint32_t n_pairs_max, const uint32_t* __restrict__ counts,
                                                             uint32_t* __restrict__ pair_key,
                                                             uint32_t* __restrict__ pair_val) {
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_d0;
    // depth ranks and pairs: the launch's bounds, or the counts on the device
    const uint32_t n = counts ? min(counts[0], n_max) : n_max;
    const uint32_t n_pairs = counts ? min(counts[1], n_pairs_max) : n_pairs_max;
    const uint32_t p0 = blockIdx.x * kEmitChunk;
    if (p0 >= n_pairs) return;
    if (threadIdx.x < 64) {
        // last d with offsets[d] <= p0 (offsets[0] == 0 <= p0; offsets never
        // decrease): a 64-way search by the first wave, one probe per lane,
        // so the chain of dependent loads is log64(n) long, not log2(n)
        const int lane = threadIdx.x;
        uint32_t lo = 0, hi = n;      // invariant: offsets[lo] <= p0, answer in [lo, hi)
        while (hi - lo > 1) {
            const uint32_t step = (hi - lo + 63) / 64;
            const uint32_t q = lo + (uint32_t)lane * step;
            const bool le = lane == 0 || (q < hi && offsets[q] <= p0);
            const unsigned long long m = __ballot(le);      // lanes 0 .. L hold: offsets are sorted
            const uint32_t L = 63u - (uint32_t)__clzll(m);
            const uint32_t nlo = lo + L * step;
            hi = min(hi, nlo + step);
            lo = nlo;
        }
        if (lane == 0) s_d0 = lo;
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
        uint32_t local = p - s_off[lo];
        const uint2 rs = rect_s[d];
        const uint32_t w = rs.y & 0xFFFFu, tw = rs.y >> 16;
        if (mask_s) {
            // the local-th covered tile of the rectangle (row-major bits)
            const uint64_t m = mask_s[d];
            if (m) local = nth_set_bit(m, local);
        }
        const uint32_t row = local / w, col = local - row * w;
        pair_key[p] = rs.x + row * tw + col;
        pair_val[p] = sorted_slot[d];
    }
}

// kRangePer pairs per thread, kRangeThreads apart (coalesced), so that each
// wave keeps several loads in flight instead of one round trip per wave
constexpr int kRangeThreads = 256, kRangePer = 4;

__global__ __launch_bounds__(kRangeThreads) void k_tile_ranges(const uint32_t* __restrict__ keys, uint32_t n_max,
                                                               const uint32_t* __restrict__ counts,
                                                               uint2* __restrict__ ranges, uint32_t n_tiles) {
    const uint32_t n = counts ? min(counts[1], n_max) : n_max;
    const uint32_t base = blockIdx.x * (kRangeThreads * kRangePer) + threadIdx.x;
#pragma unroll
    for (int j = 0; j < kRangePer; ++j) {
        const uint32_t p = base + j * kRangeThreads;
        if (p >= n) break;
        const uint32_t k = keys[p];
        if (k >= n_tiles) continue;     // keys are tile ids by construction; guards the write
        if (p == 0 || keys[p - 1] != k) ranges[k].x = p;
        if (p == n - 1 || keys[p + 1] != k) ranges[k].y = p + 1;
    }
}

// The binning's sizes from the visibility scan: visible slots (total[0]) and
// pairs (the sum of kBinPairParts partial sums, 16 apart).  The pair count
// goes to n_pairs_out; the effective counts counts[0] (visible) and
// counts[1] (pairs), read by the launches after this one, are 0 when the
// pairs exceed the capacity or 32-bit indexing, so those launches then
// produce empty lists and the caller learns of it from the count alone.
__global__ void k_bin_counts(const unsigned long long* __restrict__ total,
                             const unsigned long long* __restrict__ parts, unsigned long long capacity,
                             int64_t* __restrict__ n_pairs_out, uint32_t* __restrict__ counts) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long P = 0;
    for (int k = 0; k < kBinPairParts; ++k) P += parts[16 * k];
    const unsigned long long V = total[0];
    const bool ok = P <= capacity && P <= 0xFFFFFF00ull;
    counts[0] = ok ? (uint32_t)V : 0u;
    counts[1] = ok ? (uint32_t)P : 0u;
    *n_pairs_out = (int64_t)P;
}

// Launch order of the tiles for compositing: longest lists first, so that
// the slowest workgroups start early instead of forming the tail of the
// launch (longest-processing-time-first list scheduling).  One workgroup:
// tiles are bucketed by 1/8-octave steps of their list length (LDS counts),
// the buckets are scanned from the longest down, and every tile takes the
// next place of its bucket.  Order inside a bucket is arbitrary; results do
// not depend on it.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 256;

__device__ __forceinline__ int order_bucket(const uint2 r) {
    const uint32_t len = r.y - r.x;
    const int b = (int)(8.0f * __log2f((float)len + 1.0f));
    return kOrderBuckets - 1 - min(b, kOrderBuckets - 1);   // longest first
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                              uint32_t* __restrict__ order) {
    __shared__ uint32_t s_cnt[kOrderBuckets];
    const int tid = threadIdx.x;
    for (int b = tid; b < kOrderBuckets; b += kOrderThreads) s_cnt[b] = 0;
    __syncthreads();
    for (uint32_t t = tid; t < n_tiles; t += kOrderThreads) atomicAdd(&s_cnt[order_bucket(ranges[t])], 1u);
    __syncthreads();
    static_assert(kOrderBuckets == 256, "one wave scans the buckets, four per lane");
    if (tid < 64) wave_excl_scan256(s_cnt);
    __syncthreads();
    for (uint32_t t = tid; t < n_tiles; t += kOrderThreads) {
        const uint32_t at = atomicAdd(&s_cnt[order_bucket(ranges[t])], 1u);
        order[at] = t;
    }
}

}  // namespace

hipError_t launch_tile_order(const uint32_t* ranges, uint32_t n_tiles, uint32_t* order, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, s, reinterpret_cast<const uint2*>(ranges),
                       n_tiles, order);
    return hipGetLastError();
}

hipError_t launch_compact_visible(const Projected& proj, const uint32_t* pos, uint32_t n_slots, uint32_t* keys,
                                  uint32_t* vals, uint4* desc, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_visible, dim3((n_slots + 255) / 256), dim3(256), 0, s, proj.tiles, pos, proj.dkey,
                       proj.rect, proj.tile_mask, n_slots, keys, vals, desc);
    return hipGetLastError();
}

hipError_t launch_gather_sorted(const uint32_t* sorted_pos, const uint4* desc, uint32_t n_visible, const uint32_t* counts,
                                uint32_t* tiles_s, uint2* rect_s, uint64_t* mask_s, uint32_t* slot_s, hipStream_t s) {
    if (!n_visible) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sorted, dim3((n_visible + 255) / 256), dim3(256), 0, s, sorted_pos, desc, n_visible,
                       counts, tiles_s, rect_s, mask_s, slot_s);
    return hipGetLastError();
}

hipError_t launch_emit_pairs(const uint32_t* offsets, const uint2* rect_s, const uint64_t* mask_s,
                             const uint32_t* sorted_slot, uint32_t n_slots, uint32_t n_pairs, const uint32_t* counts,
                             uint32_t* pair_key, uint32_t* pair_val, hipStream_t s) {
    if (!n_pairs || !n_slots) return hipSuccess;
    const uint32_t blocks = (n_pairs + kEmitChunk - 1) / kEmitChunk;
    hipLaunchKernelGGL(k_emit_pairs, dim3(blocks), dim3(kEmitThreads), 0, s, offsets, rect_s, mask_s, sorted_slot,
                       n_slots, n_pairs, counts, pair_key, pair_val);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* sorted_keys, uint32_t n_pairs, const uint32_t* counts, uint32_t* ranges,
                              uint32_t n_tiles, hipStream_t s) {
    hipError_t e = fill_u32(ranges, 0u, (size_t)n_tiles * 2, s);
    if (e != hipSuccess || !n_pairs) return e;
    constexpr uint32_t per_block = kRangeThreads * kRangePer;
    hipLaunchKernelGGL(k_tile_ranges, dim3((n_pairs + per_block - 1) / per_block), dim3(kRangeThreads), 0, s,
                       sorted_keys, n_pairs, counts, reinterpret_cast<uint2*>(ranges), n_tiles);
    return hipGetLastError();
}

hipError_t launch_bin_counts(const unsigned long long* total, const unsigned long long* parts,
                             unsigned long long capacity, int64_t* n_pairs_out, uint32_t* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_bin_counts, dim3(1), dim3(64), 0, s, total, parts, capacity, n_pairs_out, counts);
    return hipGetLastError();
}

}  // namespace gs
