// Device-wide primitives for binning: a stable LSD radix sort of
// (uint32 key, uint32 value) pairs and an exclusive scan of uint32 -- gfx950.
//
// Radix pass = three steps, four launches (reduce-then-scan, no
// inter-workgroup waiting, so no kernel can hang on a missing predecessor):
//   1. upsweep: each workgroup counts the digits of its tile (1024 or 2048
//      keys); counts go to a digit-major table hist[digit][tile];
//   2. the table is exclusive-scanned in digit-major order (two launches),
//      which yields the global output offset of every (digit, tile);
//   3. downsweep: each wave64 ranks its keys in rounds of 64 with
//      ballot-based digit matching (lanes with equal digits find each other
//      through one __ballot per digit bit; rank = popcount of lower peers),
//      keeping per-wave running digit counters in LDS.  Keys and values are
//      then scattered into LDS in digit order and written out in runs, so
//      global stores are contiguous per digit.
// Stability: inside a wave items are ranked in (round, lane) order, waves
// and tiles are concatenated in order, so equal keys keep input order.
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kSortThreads = 256;
constexpr int kMaxRadixBits = 8;
// Keys per workgroup: small sorts take 4 per thread (1024 per workgroup),
// so that a sort of ~1M keys still spreads over ~1000 workgroups; larger
// ones take 8 (fewer digit-table entries to scan).
constexpr uint32_t kSmallSortMax = 1u << 21;
constexpr int kMinSortTile = kSortThreads * 4;      // digit tables are sized for this

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const unsigned lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Mask of the active lanes whose `digit` equals this lane's, restricted to
// lanes where `valid` holds.  `bits` ballots.
__device__ __forceinline__ unsigned long long match_digit(uint32_t digit, bool valid, int bits) {
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const bool bit = (digit >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// n_dev (nullable): the key count on the device, at most n (the launch's bound)
__device__ __forceinline__ uint32_t count_of(uint32_t n, const uint32_t* __restrict__ n_dev) {
    return n_dev ? min(*n_dev, n) : n;
}

// The element count of a scan over a table derived from a device count:
// ceil(*n_dev / div) * mul (the digit table of a sort: tiles x radix), at
// most n; n itself without n_dev.
__device__ __forceinline__ uint32_t scaled_count_of(uint32_t n, const uint32_t* __restrict__ n_dev, uint32_t div,
                                                    uint32_t mul) {
    if (!n_dev) return n;
    const uint64_t c = ((uint64_t)*n_dev + div - 1) / div * mul;
    return c < n ? (uint32_t)c : n;
}

template <int kSortIpt>
__global__ __launch_bounds__(kSortThreads) void k_radix_upsweep(const uint32_t* __restrict__ keys, uint32_t n_max,
                                                                const uint32_t* __restrict__ n_dev, int shift,
                                                                int bits, uint32_t* __restrict__ hist,
                                                                uint32_t n_tiles) {
    constexpr int kSortTile = kSortThreads * kSortIpt, kWaveItems = 64 * kSortIpt;
    __shared__ uint32_t cnt[4][1 << kMaxRadixBits];
    // the digit table has one column per tile that holds keys: its row
    // stride is the tile count of the device count, and workgroups past it
    // write nothing
    const uint32_t n = count_of(n_max, n_dev);
    const uint32_t n_tab = (uint32_t)(((uint64_t)n + kSortTile - 1) / kSortTile);
    if (blockIdx.x >= n_tab) return;
    (void)n_tiles;
    const int radix = 1 << bits;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // rows are (1 << kMaxRadixBits) apart: clear the whole table, not 4 * radix entries
    for (int i = threadIdx.x; i < 4 * (1 << kMaxRadixBits); i += kSortThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile + wave * kWaveItems;
    const uint32_t mask = (uint32_t)radix - 1;
    for (int r = 0; r < kSortIpt; ++r) {
        const uint32_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t d = valid ? (keys[idx] >> shift) & mask : 0u;
        const unsigned long long m = match_digit(d, valid, bits);
        if (valid && lane == __ffsll((unsigned long long)m) - 1) cnt[wave][d] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < radix; d += kSortThreads)
        hist[(size_t)d * n_tab + blockIdx.x] = cnt[0][d] + cnt[1][d] + cnt[2][d] + cnt[3][d];
}

template <int kSortIpt>
__global__ __launch_bounds__(kSortThreads) void k_radix_downsweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, uint32_t n_max, const uint32_t* __restrict__ n_dev, int shift, int bits,
    const uint32_t* __restrict__ hist_scan, uint32_t n_tiles) {
    constexpr int kSortTile = kSortThreads * kSortIpt, kWaveItems = 64 * kSortIpt;
    const uint32_t n = count_of(n_max, n_dev);
    if (blockIdx.x * (uint32_t)kSortTile >= n) return;     // no keys in this tile
    const uint32_t n_tab = (uint32_t)(((uint64_t)n + kSortTile - 1) / kSortTile);   // digit-table stride
    (void)n_tiles;
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t s_wcnt[4][1 << kMaxRadixBits];
    __shared__ uint32_t s_bstart[1 << kMaxRadixBits];
    __shared__ uint32_t s_goff[1 << kMaxRadixBits];
    __shared__ uint32_t s_wsum[4];

    const int radix = 1 << bits;
    const uint32_t mask = (uint32_t)radix - 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < 4 * (1 << kMaxRadixBits); i += kSortThreads) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();

    const uint32_t tile0 = blockIdx.x * kSortTile;
    const uint32_t base = tile0 + wave * kWaveItems;
    uint32_t key[kSortIpt], val[kSortIpt], rank[kSortIpt];
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
        const uint32_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : 0u;
        val[r] = valid ? vin[idx] : 0u;
    }
    const unsigned long long lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
        const uint32_t idx = base + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t d = (key[r] >> shift) & mask;
        const unsigned long long m = match_digit(d, valid, bits);
        uint32_t pre = 0;
        if (valid) pre = s_wcnt[wave][d];
        rank[r] = pre + (uint32_t)__popcll(m & lt);
        // every lane of the wave reads the counter before the group leader
        // rewrites it: one wave's LDS instructions execute in order; the
        // wave barrier keeps the compiler from moving LDS accesses across
        __builtin_amdgcn_wave_barrier();
        if (valid && lane == __ffsll((unsigned long long)m) - 1) s_wcnt[wave][d] = pre + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // per digit: exclusive prefix over waves, block total, then an exclusive
    // scan of the block totals over digits
    uint32_t total = 0;
    if ((int)threadIdx.x < radix) {
        const int d = threadIdx.x;
        const uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
        s_wcnt[0][d] = 0;
        s_wcnt[1][d] = c0;
        s_wcnt[2][d] = c0 + c1;
        s_wcnt[3][d] = c0 + c1 + c2;
        total = c0 + c1 + c2 + c3;
        s_goff[d] = hist_scan[(size_t)d * n_tab + blockIdx.x];
    }
    // block-wide exclusive scan of `total` (thread d holds digit d)
    uint32_t incl = total;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += s_wsum[w];
    if ((int)threadIdx.x < radix) s_bstart[threadIdx.x] = wpre + incl - total;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
        const uint32_t idx = base + r * 64 + lane;
        if (idx < n) {
            const uint32_t d = (key[r] >> shift) & mask;
            const uint32_t lp = s_bstart[d] + s_wcnt[wave][d] + rank[r];
            s_keys[lp] = key[r];
            s_vals[lp] = val[r];
        }
    }
    __syncthreads();
    const uint32_t count = min((uint32_t)kSortTile, n - tile0);
    for (uint32_t i = threadIdx.x; i < count; i += kSortThreads) {
        const uint32_t k = s_keys[i];
        const uint32_t d = (k >> shift) & mask;
        const uint32_t gp = s_goff[d] + (i - s_bstart[d]);
        if (gp < n) {     // always true for a consistent histogram; guards the write
            kout[gp] = k;
            vout[gp] = s_vals[i];
        }
    }
}

// ---------------------------------------------------------------- scan

constexpr int kScanThreads = 256;
constexpr int kScanSumParts = kBinPairParts;
constexpr int kScanIpt = 16;
constexpr int kScanTile = kScanThreads * kScanIpt;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// tile sums
// The scanned value of element i: in[i], or with kFlags, 1 where in[i] != 0.
template <bool kFlags>
__device__ __forceinline__ uint32_t scan_value(uint32_t x) {
    return kFlags ? (x != 0u ? 1u : 0u) : x;
}

// Tile sums.  With kFlags the raw values are also summed (64-bit) into
// kScanSumParts counters 16 apart (one atomic address would serialise
// thousands of workgroups from all XCDs); the counters must start at 0.
template <bool kFlags>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, uint32_t n_max,
                                                              const uint32_t* __restrict__ n_dev, uint32_t div,
                                                              uint32_t mul, uint32_t* __restrict__ tsum,
                                                              unsigned long long* __restrict__ raw_parts) {
    __shared__ uint32_t s_w[4];
    __shared__ unsigned long long s_raw[4];
    const uint32_t n = scaled_count_of(n_max, n_dev, div, mul);
    // workgroups past the count exit (the first always runs)
    if (blockIdx.x > 0 && blockIdx.x * (uint32_t)kScanTile >= n) return;
    const uint32_t base = blockIdx.x * kScanTile;
    uint32_t acc = 0;
    unsigned long long raw = 0;
#pragma unroll
    for (int r = 0; r < kScanIpt; ++r) {
        const uint32_t idx = base + r * kScanThreads + threadIdx.x;
        const uint32_t x = idx < n ? in[idx] : 0u;
        acc += scan_value<kFlags>(x);
        if (kFlags) raw += x;
    }
    const uint32_t w = wave_incl_scan(acc);
    if ((threadIdx.x & 63) == 63) s_w[threadIdx.x >> 6] = w;
    if (kFlags) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) raw += __shfl_xor(raw, off, 64);
        if ((threadIdx.x & 63) == 0) s_raw[threadIdx.x >> 6] = raw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tsum[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (kFlags) {
            const unsigned long long b = s_raw[0] + s_raw[1] + s_raw[2] + s_raw[3];
            if (b) atomicAdd(&raw_parts[16 * (blockIdx.x % kScanSumParts)], b);   // one 128-byte line each
        }
    }
}

// per-tile exclusive scan plus the tile's offset; items are blocked per
// thread (16 consecutive) so that the in-thread prefix is sequential.  The
// tile's offset is the sum of the earlier tiles' sums, which every
// workgroup adds up itself (64-bit, at most a few thousand values) rather
// than waiting for a separate one-workgroup launch; the last workgroup
// that holds elements (the first, for none) writes the 64-bit total.
template <bool kFlags>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* __restrict__ in,
                                                            uint32_t* __restrict__ out, uint32_t n_max,
                                                            const uint32_t* __restrict__ n_dev, uint32_t div,
                                                            uint32_t mul, const uint32_t* __restrict__ tsum,
                                                            unsigned long long* __restrict__ total) {
    __shared__ uint32_t s_buf[kScanTile];
    const uint32_t n = scaled_count_of(n_max, n_dev, div, mul);
    const uint32_t n_act = (uint32_t)(((uint64_t)n + kScanTile - 1) / kScanTile);
    const uint32_t last_wg = n_act > 0 ? n_act - 1 : 0;
    if (blockIdx.x > last_wg) return;
    __shared__ uint32_t s_w[4];
    __shared__ unsigned long long s_off[4];
    const uint32_t base = blockIdx.x * kScanTile;
    {
        unsigned long long acc = 0;
        for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kScanThreads) acc += tsum[t];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) s_off[threadIdx.x >> 6] = acc;
    }
#pragma unroll
    for (int r = 0; r < kScanIpt; ++r) {
        const uint32_t i = r * kScanThreads + threadIdx.x;
        s_buf[i] = (base + i < n) ? scan_value<kFlags>(in[base + i]) : 0u;
    }
    __syncthreads();
    uint32_t v[kScanIpt];
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < kScanIpt; ++r) {
        v[r] = s_buf[threadIdx.x * kScanIpt + r];
        acc += v[r];
    }
    const uint32_t incl = wave_incl_scan(acc);
    if ((threadIdx.x & 63) == 63) s_w[threadIdx.x >> 6] = incl;
    __syncthreads();
    const unsigned long long tile_off = s_off[0] + s_off[1] + s_off[2] + s_off[3];
    if (blockIdx.x == last_wg && threadIdx.x == 0) *total = tile_off + tsum[blockIdx.x];
    uint32_t pre = (uint32_t)tile_off + incl - acc;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) pre += s_w[w];
#pragma unroll
    for (int r = 0; r < kScanIpt; ++r) {
        s_buf[threadIdx.x * kScanIpt + r] = pre;
        pre += v[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScanIpt; ++r) {
        const uint32_t i = r * kScanThreads + threadIdx.x;
        if (base + i < n) out[base + i] = s_buf[i];
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

size_t radix_hist_elems(uint32_t n) {
    // sized for the smallest tile, so that the size grows with n
    const size_t tiles = (n + kMinSortTile - 1) / kMinSortTile;
    return (tiles ? tiles : 1) * (size_t)(1 << kMaxRadixBits) + scan_tmp_elems((uint32_t)(tiles * 256));
}

// tile sums, padded to an even count, then the 64-bit total
static size_t scan_sums_elems(uint32_t n) {
    const size_t t = (n + kScanTile - 1) / kScanTile;
    return ((t ? t : 1) + 1) & ~size_t(1);
}

size_t scan_tmp_elems(uint32_t n) { return scan_sums_elems(n) + 2; }

hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tmp,
                              unsigned long long* total, hipStream_t s, const uint32_t* n_dev, uint32_t div,
                              uint32_t mul) {
    const uint32_t nt = (n + kScanTile - 1) / kScanTile;
    if (n == 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)total, 0u, (size_t)2);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce<false>, dim3(nt), dim3(kScanThreads), 0, s, in, n, n_dev, div, mul, tmp,
                       (unsigned long long*)nullptr);
    hipLaunchKernelGGL(k_scan_down<false>, dim3(nt), dim3(kScanThreads), 0, s, in, out, n, n_dev, div, mul, tmp,
                       total);
    return hipGetLastError();
}

hipError_t exclusive_scan_nonzero_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tmp,
                                      unsigned long long* total, unsigned long long* sum_parts, hipStream_t s) {
    const uint32_t nt = (n + kScanTile - 1) / kScanTile;
    if (n == 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)total, 0u, (size_t)2);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce<true>, dim3(nt), dim3(kScanThreads), 0, s, in, n, (const uint32_t*)nullptr, 1u,
                       1u, tmp, sum_parts);
    hipLaunchKernelGGL(k_scan_down<true>, dim3(nt), dim3(kScanThreads), 0, s, in, out, n, (const uint32_t*)nullptr,
                       1u, 1u, tmp, total);
    return hipGetLastError();
}

int radix_passes(uint32_t n, int begin_bit, int end_bit) {
    return (n <= 1 || end_bit <= begin_bit) ? 0 : (end_bit - begin_bit + kMaxRadixBits - 1) / kMaxRadixBits;
}

// Sorts keys/vals on bits [begin_bit, end_bit) with passes of <= 8 bits of
// near-equal width.  The result lands in (keys, vals) or in the alternate
// buffers; *result_in_alt says which.  `hist` needs radix_hist_elems(n).
// With n_dev the key count is read on the device (at most n, which sizes
// the launches), so the sort needs no host knowledge of it: the digit
// table and its scan cover only the tiles that hold keys.  small_tiles
// forces 1024-key tiles (for a device count expected well below n).
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t n,
                            int begin_bit, int end_bit, uint32_t* hist, hipStream_t s, bool* result_in_alt,
                            const uint32_t* n_dev, bool small_tiles) {
    *result_in_alt = false;
    if (radix_passes(n, begin_bit, end_bit) == 0) return hipSuccess;
    const int total_bits = end_bit - begin_bit;
    const int passes = (total_bits + kMaxRadixBits - 1) / kMaxRadixBits;
    const bool small = small_tiles || n <= kSmallSortMax;
    const uint32_t sort_tile = (uint32_t)kSortThreads * (small ? 4u : 8u);
    const uint32_t tiles = (n + sort_tile - 1) / sort_tile;
    const size_t hist_elems = (size_t)tiles * (1 << kMaxRadixBits);
    uint32_t* scan_tmp = hist + hist_elems;
    unsigned long long* total = reinterpret_cast<unsigned long long*>(scan_tmp + scan_sums_elems((uint32_t)hist_elems));
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    int shift = begin_bit;
    for (int p = 0; p < passes; ++p) {
        const int remaining = end_bit - shift;
        const int bits = (remaining + (passes - p) - 1) / (passes - p);
        const uint32_t radix_elems = (uint32_t)tiles << bits;
        if (small)
            hipLaunchKernelGGL(k_radix_upsweep<4>, dim3(tiles), dim3(kSortThreads), 0, s, ki, n, n_dev, shift, bits,
                               hist, tiles);
        else
            hipLaunchKernelGGL(k_radix_upsweep<8>, dim3(tiles), dim3(kSortThreads), 0, s, ki, n, n_dev, shift, bits,
                               hist, tiles);
        hipError_t e = exclusive_scan_u32(hist, hist, radix_elems, scan_tmp, total, s, n_dev, sort_tile, 1u << bits);
        if (e != hipSuccess) return e;
        if (small)
            hipLaunchKernelGGL(k_radix_downsweep<4>, dim3(tiles), dim3(kSortThreads), 0, s, ki, vi, ko, vo, n, n_dev,
                               shift, bits, hist, tiles);
        else
            hipLaunchKernelGGL(k_radix_downsweep<8>, dim3(tiles), dim3(kSortThreads), 0, s, ki, vi, ko, vo, n, n_dev,
                               shift, bits, hist, tiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        shift += bits;
        uint32_t* t;
        t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        *result_in_alt = !*result_in_alt;
    }
    return hipSuccess;
}

}  // namespace gs
