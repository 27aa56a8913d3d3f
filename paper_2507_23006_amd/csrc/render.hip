// Front-to-back compositing (Eq. 2) and its backward -- gfx950.
//
// Four wave64s per 16x16 tile, each owning an 8x8 quadrant (one pixel per
// lane) and walking the tile's depth-ordered list independently.  Records
// are staged in LDS in chunks of 64, culled against the quadrant with each
// record's alpha box and compacted by ballot; all lanes then read the same
// staged record, which the LDS serves as a broadcast.  The forward keeps no
// per-pixel lists: it stores the final transmittance and the position of the
// last composited entry, and the backward walks the list back to front,
// recovering T_i = T_{i+1} / (1 - alpha_i).
//
// Backward per entry: the 12 gradient fields are summed over the wave by
// halving lane exchanges (permlane swaps, then DPP row shifts) into an LDS
// row; after each chunk the wave adds the rows to the per-slot 2D gradient
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

// Four independent wave64s per 16x16 tile, one 8x8 quadrant each, one
// pixel per lane.  A wave walks the tile's list in chunks of 64: every lane
// gathers one record, tests the record's box (opacity' G' >= 1/255 region,
// with margins) against the wave's quadrant, and the ballot of survivors
// compacts them, in list order, into the wave's LDS slice.  The wave then
// evaluates only the survivors: an entry whose box misses every pixel of the
// quadrant has alpha < 1/255 there and would be skipped anyway, so results
// are unchanged while the horizon tiles' long lists of tiny, distant
// Gaussians cost a fraction of the work.  The per-entry update is predicated
// (selects, no branches).  Waves of a tile never wait for each other.
constexpr int kChunk = 64;
constexpr int kWaves = 4;

// the workgroup's tile: its place in the launch order (an order that is not
// a permutation of the tiles falls back to the index, so no access strays)
__device__ __forceinline__ int launch_tile(const uint32_t* __restrict__ tile_order, const ViewTable& vt) {
    const uint32_t t = tile_order ? tile_order[blockIdx.x] : blockIdx.x;
    return t < (uint32_t)vt.total_tiles ? (int)t : (int)blockIdx.x;
}

struct PixelCoords {
    int v;
    float ox, oy;          // tile origin in pixels
    float fpx, fpy;        // pixel centre relative to the tile origin
    float qcx, qcy;        // centre of the wave's quadrant (pixel-centre span +-3.5)
    bool inside;
    int64_t pix;
    int lx, ly;            // pixel within the tile
};

__device__ __forceinline__ PixelCoords pixel_coords(const ViewTable& vt, int tile, int wave, int lane) {
    PixelCoords c;
    c.v = view_of_tile(vt, tile);
    const ViewK& V = vt.v[c.v];
    const int lt = tile - V.tile_off;
    const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
    const int qx0 = (wave & 1) * 8, qy0 = (wave >> 1) * 8;
    const int lx = qx0 + (lane & 7), ly = qy0 + (lane >> 3);
    c.ox = (float)(tx * kTile);
    c.oy = (float)(ty * kTile);
    c.fpx = (float)lx + 0.5f;
    c.fpy = (float)ly + 0.5f;
    c.qcx = (float)qx0 + 4.0f;
    c.qcy = (float)qy0 + 4.0f;
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    c.inside = px < V.W && py < V.H;
    c.pix = V.pix_off + (int64_t)py * V.W + px;
    c.lx = lx;
    c.ly = ly;
    return c;
}

// does the record's alpha box reach the wave's quadrant of pixel centres?
__device__ __forceinline__ bool box_hits_quadrant(const float4 g, const float4 r3, float qcx, float qcy) {
    const float mx = g.x, my = g.y;
    return fabsf(mx - qcx) <= r3.x + 3.5f + 1e-3f + 1e-6f * fabsf(mx) &&
           fabsf(my - qcy) <= r3.y + 3.5f + 1e-3f + 1e-6f * fabsf(my) && r3.x >= 0.0f;
}

// Does the entry's alpha reach 1/255 anywhere in the wave's quadrant?  The
// exponent p(d) = qa dx^2 + qb dx dy + qc dy^2 (d = pixel centre - mean) is a
// concave quadratic; its maximum over the rectangle spanned by the
// quadrant's pixel centres is 0 when the mean lies inside, otherwise the
// largest of the four edges' one-dimensional maxima.  The entry can only be
// composited where o' 2^p >= 1/255, i.e. p >= log2(1/(255 o')); the test is
// relaxed by 1e-5 and by 16 float32 ulps of the terms' magnitudes, which
// covers the rounding of both this test and the kernels' own evaluation of
// p, so an entry it rejects has alpha < 1/255 at every pixel of the quadrant.
__device__ __forceinline__ float edge_max(float qa, float qb, float qc, float dx, float lo, float hi) {
    // max over dy in [lo, hi] of qa dx^2 + qb dx dy + qc dy^2 (qc < 0)
    const float dy = fminf(fmaxf(-qb * dx / (2.0f * qc), lo), hi);
    return fmaf(qa, dx * dx, fmaf(qb, dx * dy, qc * (dy * dy)));
}

__device__ __forceinline__ bool ellipse_hits_quadrant(const float4 g, const float4 r1, float qcx, float qcy) {
    const float qa = g.z, qb = g.w, qc = r1.x, o = r1.y;
    const float dx0 = (qcx - 3.5f) - g.x, dx1 = (qcx + 3.5f) - g.x;
    const float dy0 = (qcy - 3.5f) - g.y, dy1 = (qcy + 3.5f) - g.y;
    if (dx0 <= 0.0f && dx1 >= 0.0f && dy0 <= 0.0f && dy1 >= 0.0f) return true;
    float m = fmaxf(edge_max(qa, qb, qc, dx0, dy0, dy1), edge_max(qa, qb, qc, dx1, dy0, dy1));
    m = fmaxf(m, fmaxf(edge_max(qc, qb, qa, dy0, dx0, dx1), edge_max(qc, qb, qa, dy1, dx0, dx1)));
    const float DX = fmaxf(fabsf(dx0), fabsf(dx1)), DY = fmaxf(fabsf(dy0), fabsf(dy1));
    const float mag = fabsf(qa) * DX * DX + fabsf(qb) * DX * DY + fabsf(qc) * DY * DY;
    const float thr = -__log2f(255.0f * o) - 1e-5f - 16.0f * 5.9604645e-8f * mag;
    return m >= thr;
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

struct WaveStage {
    float4 g[kChunk];      // tile-relative mean, qa, qb
    float4 b[kChunk];      // qc, opacity', depth, 2 qc
    float4 c[kChunk];      // r, g, b, 2 qa
    int4 ps[kChunk];       // 1-based position in the tile list, slot, -, - (16-byte stride like the
                           // records, so one address register serves every per-entry read)
};

// Gathers list entries [j0, j0 + 64) of the tile (clipped to `end`), keeps
// those whose box reaches the quadrant, compacts them in order into `st`;
// returns the number kept.  Wave-uniform.
__device__ __forceinline__ int stage_chunk(const float4* __restrict__ rec, const uint32_t* __restrict__ pair_vals,
                                           uint32_t list0, uint32_t j0, uint32_t end, const PixelCoords& pc,
                                           int lane, WaveStage& st) {
    const uint32_t j = j0 + lane;
    bool hit = false;
    float4 g, r1, r2;
    uint32_t s = 0;
    if (j < end) {
        s = pair_vals[j];
        const float4 r0 = rec[4 * (size_t)s + 0];
        r1 = rec[4 * (size_t)s + 1];
        r2 = rec[4 * (size_t)s + 2];
        const float4 r3 = rec[4 * (size_t)s + 3];
        g = stage_geom(r0, r1, r2, pc.ox, pc.oy);
        hit = box_hits_quadrant(g, r3, pc.qcx, pc.qcy);
    }
    const unsigned long long m = __ballot(hit);
    if (hit) {
        const int d = __popcll(m & lanes_below(lane));
        st.g[d] = g;
        st.b[d] = r1;
        st.c[d] = r2;
        st.ps[d] = make_int4((int)(j - list0) + 1, (int)s, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
    return __popcll(m);
}

// largest i in [0, n] with a[i] <= v (a non-decreasing, a[0] <= v)
__device__ __forceinline__ uint32_t last_le(const uint32_t* __restrict__ a, uint32_t n, uint32_t v) {
    uint32_t lo = 0, hi = n + 1;      // invariant: a[lo] <= v, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// tile at launch position i (the order, when valid, else the position)
__device__ __forceinline__ int order_tile(const uint32_t* __restrict__ tile_order, const ViewTable& vt, uint32_t i) {
    const uint32_t t = tile_order ? tile_order[i] : i;
    return t < (uint32_t)vt.total_tiles ? (int)t : (int)i;
}

// One lane's list entry, loaded a chunk ahead of its use so that the two
// dependent gathers (pair value, then record) overlap the evaluation of the
// previous chunk instead of stalling the wave.  Staging marks the fourth
// record's unused lanes (z, w) as read: registers of a pending load that
// the compiler sees as dead get reused as temporaries, which makes the wave
// wait for the load at once.
struct Gather {
    float4 r0, r1, r2, r3;
    uint32_t slot;
};

constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t load_slot(const uint32_t* __restrict__ pair_vals, uint32_t j, uint32_t end) {
    return j < end ? pair_vals[j] : kNoSlot;
}

__device__ __forceinline__ Gather load_entry(const float4* __restrict__ rec, uint32_t s) {
    Gather g;
    g.slot = s;
    if (s != kNoSlot) {
        g.r0 = rec[4 * (size_t)s + 0];
        g.r1 = rec[4 * (size_t)s + 1];
        g.r2 = rec[4 * (size_t)s + 2];
        g.r3 = rec[4 * (size_t)s + 3];
    } else {
        g.r0 = g.r1 = g.r2 = g.r3 = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
    }
    return g;
}

// box test, ballot and in-order compaction of a gathered chunk into `st`;
// pos = the lane's 1-based position in the tile list.  Wave-uniform result.
__device__ __forceinline__ int stage_gathered(const Gather& e, int pos, const PixelCoords& pc, int lane,
                                              WaveStage& st) {
    __asm__ volatile("" ::"v"(e.r3.z), "v"(e.r3.w));   // emits no instruction
    const float4 g = stage_geom(e.r0, e.r1, e.r2, pc.ox, pc.oy);
    const bool hit = e.slot != kNoSlot && box_hits_quadrant(g, e.r3, pc.qcx, pc.qcy) &&
                     ellipse_hits_quadrant(g, e.r1, pc.qcx, pc.qcy);
    const unsigned long long m = __ballot(hit);
    if (hit) {
        const int d = __popcll(m & lanes_below(lane));
        st.g[d] = g;
        st.b[d] = make_float4(e.r1.x, e.r1.y, e.r1.z, 2.0f * e.r1.x);
        st.c[d] = make_float4(e.r2.x, e.r2.y, e.r2.z, 2.0f * g.z);
        st.ps[d] = make_int4(pos, (int)e.slot, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
    return __popcll(m);
}

// segmented forward: stop_seg value of a pixel still compositing after
// the head; segments in the head (walked by the tile's workgroup)
constexpr int32_t kSegAlive = 0x7fffffff;
constexpr int kHeadSegs = 2;

// One wave composites quadrant `quad` of `tile` (staging in its LDS slice
// `st`) and writes its pixels: the whole list, front to back.  With
// head_stop (the tile's stop_seg row; a list the plan segments) only the
// head, the first kHeadSegs segments: pixels that stop there (or whose list
// ends there) get their outputs and stop_seg = -1, the others their state
// after it (rgb without background, depth, T, last) and stop_seg =
// kSegAlive.  The head also writes the backward's states of its segments
// 1 .. kHeadSegs - 1 (head_states: the tile's first stored state) from the
// pixel's (T, C, D) at the segment's ends: T_seg = T_end / T_start and
// C_seg = (C_end - C_start) / T_start -- the segment's composite with T
// restarted at 1; the backward uses C_seg scaled back by T_start, so the
// subtraction's rounding stays at the size of C's.
__device__ __forceinline__ void render_fwd_quadrant(const float4* __restrict__ rec,
                                                    const uint32_t* __restrict__ pair_vals,
                                                    const uint2* __restrict__ ranges, const ViewTable& vt,
                                                    const OptK& opt, int tile, int quad, int lane, WaveStage& st,
                                                    float* __restrict__ rgb, float* __restrict__ depth,
                                                    float* __restrict__ alpha_out, float* __restrict__ T_out,
                                                    int32_t* __restrict__ last_out,
                                                    int32_t* __restrict__ head_stop = nullptr,
                                                    float* __restrict__ head_states = nullptr) {
    const PixelCoords pc = pixel_coords(vt, tile, quad, lane);
    const uint2 rg = ranges[tile];
    const uint32_t end = head_stop ? min(rg.x + (uint32_t)(kHeadSegs * kSegLen), rg.y) : rg.y;

    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, D = 0.0f;
    int last = 0;
    bool alive = pc.inside;
    // (T, C, D) at the start of the current segment (head walks only)
    float sT = 1.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, sD = 0.0f;
    int seg = 0;
    const int px = pc.ly * kTile + pc.lx;
    auto seg_state = [&]() {      // state of segment `seg` >= 1 from its start to now
        float* o = head_states + (size_t)(seg - 1) * kSegFields * 256;
        const float inv = 1.0f / sT;
        o[0 * 256 + px] = T * inv;
        o[1 * 256 + px] = (c0 - s0) * inv;
        o[2 * 256 + px] = (c1 - s1) * inv;
        o[3 * 256 + px] = (c2 - s2) * inv;
        o[4 * 256 + px] = (D - sD) * inv;
    };
    Gather cur = load_entry(rec, load_slot(pair_vals, rg.x + lane, end));
    uint32_t s_next = load_slot(pair_vals, rg.x + kChunk + lane, end);
    for (uint32_t j0 = rg.x; j0 < end; j0 += kChunk) {
        if (head_states && j0 != rg.x && (j0 - rg.x) % (uint32_t)kSegLen == 0) {
            if (seg >= 1) seg_state();
            ++seg;
            sT = T;
            s0 = c0;
            s1 = c1;
            s2 = c2;
            sD = D;
        }
        if (__ballot(alive) == 0) break;     // every pixel of the quadrant has stopped
        const int n = stage_gathered(cur, (int)(j0 - rg.x) + lane + 1, pc, lane, st);
        cur = load_entry(rec, s_next);                                   // next chunk's records
        s_next = load_slot(pair_vals, j0 + 2 * kChunk + lane, end);      // and the one after's slots
        // entry k + 1 is read from LDS while entry k is evaluated; the
        // position of the pixel's last composited entry is read once per chunk
        int last_k = -1;
        float4 an = st.g[0], bn = st.b[0], cn = st.c[0];
#pragma unroll 4
        for (int k = 0; k < n; ++k) {
            const float4 a = an, b = bn, c = cn;
            const int kn = k + 1 < n ? k + 1 : k;
            an = st.g[kn];
            bn = st.b[kn];
            cn = st.c[kn];
            const Eval e = eval_entry(a, b, pc.fpx, pc.fpy);
            const float Tn = T * (1.0f - e.alpha);
            const bool keep = alive && e.keep;
            const bool stop = keep && Tn < kTMin;
            const bool use = keep && !stop;
            const float w = use ? e.alpha * T : 0.0f;
            c0 = fmaf(c.x, w, c0);
            c1 = fmaf(c.y, w, c1);
            c2 = fmaf(c.z, w, c2);
            D = fmaf(b.z, w, D);
            T = use ? Tn : T;
            last_k = use ? k : last_k;
            alive = alive && !stop;
        }
        if (last_k >= 0) last = st.ps[last_k].x;
        __builtin_amdgcn_wave_barrier();     // the chunk is consumed before the next one is staged
    }
    if (head_states && seg >= 1) seg_state();
    if (!pc.inside) return;
    const int64_t p = pc.pix;
    const bool more = head_stop && alive && end < rg.y;    // compositing continues after the head
    if (head_stop) head_stop[px] = more ? kSegAlive : -1;
    rgb[3 * p + 0] = more ? c0 : fmaf(T, opt.bg[0], c0);
    rgb[3 * p + 1] = more ? c1 : fmaf(T, opt.bg[1], c1);
    rgb[3 * p + 2] = more ? c2 : fmaf(T, opt.bg[2], c2);
    depth[p] = D;
    if (!more) alpha_out[p] = 1.0f - T;
    T_out[p] = T;
    last_out[p] = last;
}

// Segmented forward, pass 2: one wave walks segment `seg` >= kHeadSegs
// (list positions [seg S, (seg + 1) S), S = kSegLen) of a long list for the
// pixels of its quadrant still compositing after the head (`on`),
// and keeps, over the entries that pass the alpha test, the segment's
// state with T restarted at 1: T_seg = prod (1 - alpha), C_seg = sum c
// alpha T_local (colour and depth) and the position of its last such entry
// -- as if no pixel stopped in the segment -- in its stored-state row
// (planes T, r, g, b, depth, last; the other pixels get the empty state).
// A pixel whose T_local falls below T_min is certain to stop in this
// segment or an earlier one (T before it is at most 1); it is left there
// (the fold then stops in or before this segment, whose exact walk pass 4
// redoes), and the wave stops when all its pixels are.
__device__ __forceinline__ void render_fwd_segment(const float4* __restrict__ rec,
                                                   const uint32_t* __restrict__ pair_vals, const uint2 rg,
                                                   const PixelCoords& pc, bool on, int seg, int lane, WaveStage& st,
                                                   float* __restrict__ state_row) {
    const uint32_t lo = rg.x + (uint32_t)seg * kSegLen, hi = min(lo + (uint32_t)kSegLen, rg.y);
    float Tl = 1.0f, l0 = 0.0f, l1 = 0.0f, l2 = 0.0f, Dl = 0.0f;
    int last = 0;
    Gather cur = load_entry(rec, load_slot(pair_vals, lo + lane, hi));
    uint32_t s_next = load_slot(pair_vals, lo + kChunk + lane, hi);
    for (uint32_t j0 = lo; j0 < hi; j0 += kChunk) {
        if (__ballot(on) == 0) break;
        const int n = stage_gathered(cur, (int)(j0 - rg.x) + lane + 1, pc, lane, st);
        cur = load_entry(rec, s_next);
        s_next = load_slot(pair_vals, j0 + 2 * kChunk + lane, hi);
        int last_k = -1;
#pragma unroll 4
        for (int k = 0; k < n; ++k) {
            const float4 a = st.g[k], b = st.b[k], c = st.c[k];
            const Eval e = eval_entry(a, b, pc.fpx, pc.fpy);
            const bool use = on && e.keep;
            const float w = use ? e.alpha * Tl : 0.0f;
            l0 = fmaf(c.x, w, l0);
            l1 = fmaf(c.y, w, l1);
            l2 = fmaf(c.z, w, l2);
            Dl = fmaf(b.z, w, Dl);
            Tl = use ? Tl * (1.0f - e.alpha) : Tl;
            last_k = use ? k : last_k;
        }
        if (last_k >= 0) last = st.ps[last_k].x;
        on = on && Tl >= kTMin;
        __builtin_amdgcn_wave_barrier();
    }
    const int px = pc.ly * kTile + pc.lx;
    state_row[0 * 256 + px] = Tl;
    state_row[1 * 256 + px] = l0;
    state_row[2 * 256 + px] = l1;
    state_row[3 * 256 + px] = l2;
    state_row[4 * 256 + px] = Dl;
    reinterpret_cast<int32_t*>(state_row)[5 * 256 + px] = last;
}

// stored segment b of a plan -> launch position, segment (>= 1), count
struct SegItem {
    uint32_t i;
    int seg, nseg;
};
__device__ __forceinline__ SegItem stored_seg(const SegPlan& plan, uint32_t b) {
    SegItem it;
    it.i = last_le(plan.state_off, plan.n_tiles, b);
    it.seg = (int)(b - plan.state_off[it.i]) + 1;
    it.nseg = (int)(plan.work_off[it.i + 1] - plan.work_off[it.i]);
    return it;
}

// One workgroup per tile, in launch order.  With a segment plan, the lists
// it segments composite their head only (pass 1 of the segmented forward).
// (256, 7): at most 72 VGPRs, 7 waves per SIMD, no spills.
__global__ __launch_bounds__(256, 7) void k_render_fwd(const float4* __restrict__ rec,
                                                    const uint32_t* __restrict__ pair_vals,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ tile_order, ViewTable vt, OptK opt,
                                                    float* __restrict__ rgb, float* __restrict__ depth,
                                                    float* __restrict__ alpha_out, float* __restrict__ T_out,
                                                    int32_t* __restrict__ last_out, SegPlan plan) {
    __shared__ WaveStage stage[kWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = launch_tile(tile_order, vt);
    int32_t* head_stop = nullptr;
    float* head_states = nullptr;
    if (plan.work_off) {
        const uint32_t i = blockIdx.x;
        if (plan.work_off[i + 1] - plan.work_off[i] > 1u) {
            head_stop = plan.stop_seg + (size_t)tile * 256;
            head_states = plan.state + (size_t)plan.state_off[i] * kSegFields * 256;
        }
    }
    render_fwd_quadrant(rec, pair_vals, ranges, vt, opt, tile, wave, lane, stage[wave], rgb, depth, alpha_out, T_out,
                        last_out, head_stop, head_states);
}

// Pass 2, one workgroup per stored segment: the segment's state for the
// pixels still compositing after the head (a quadrant with none exits).
// (256, 7): at most 72 VGPRs, 7 waves per SIMD, no spills.
__global__ __launch_bounds__(256, 7) void k_fwd_segments(const float4* __restrict__ rec,
                                                      const uint32_t* __restrict__ pair_vals,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ tile_order, ViewTable vt,
                                                      SegPlan plan) {
    __shared__ WaveStage stage[kWaves];
    const uint32_t b = blockIdx.x;
    if (b >= plan.state_off[plan.n_tiles]) return;
    const SegItem it = stored_seg(plan, b);
    if (it.seg < kHeadSegs) return;        // the head's segments
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = order_tile(tile_order, vt, it.i);
    const PixelCoords pc = pixel_coords(vt, tile, wave, lane);
    const bool on = pc.inside && plan.stop_seg[(size_t)tile * 256 + pc.ly * kTile + pc.lx] == kSegAlive;
    if (__ballot(on) == 0) return;
    render_fwd_segment(rec, pair_vals, ranges[tile], pc, on, it.seg, lane, stage[wave],
                       plan.state + (size_t)b * kSegFields * 256);
}

// Pass 3, one thread per pixel still compositing after the head of a
// segmented list: fold the segments after it front to back (C += T C_seg,
// T *= T_seg).  T only decreases along the list, so the pixel stops inside
// segment j exactly when T T_seg_j < T_min; then its state before segment j
// is left in the outputs and stop_seg = j for pass 4.  Otherwise the
// outputs are final and stop_seg = -1.
__global__ __launch_bounds__(256) void k_fwd_combine(const uint32_t* __restrict__ tile_order, ViewTable vt,
                                                     OptK opt, SegPlan plan, float* __restrict__ rgb,
                                                     float* __restrict__ depth, float* __restrict__ alpha_out,
                                                     float* __restrict__ T_out, int32_t* __restrict__ last_out) {
    const uint32_t i = blockIdx.x;
    const int nseg = (int)(plan.work_off[i + 1] - plan.work_off[i]);
    if (nseg <= 1) return;
    const int tile = order_tile(tile_order, vt, i);
    const PixelCoords pc = pixel_coords(vt, tile, threadIdx.x >> 6, threadIdx.x & 63);
    const int px = pc.ly * kTile + pc.lx;
    int32_t* stop_row = plan.stop_seg + (size_t)tile * 256;
    if (!pc.inside || stop_row[px] != kSegAlive) return;
    const int64_t p = pc.pix;
    float T = T_out[p], c0 = rgb[3 * p + 0], c1 = rgb[3 * p + 1], c2 = rgb[3 * p + 2], D = depth[p];
    int last = last_out[p];
    int stop = -1;
    const uint32_t st0 = plan.state_off[i];
    for (int j = kHeadSegs; j < nseg; ++j) {
        const float* r = plan.state + (size_t)(st0 + (uint32_t)(j - 1)) * kSegFields * 256;
        const float Ts = r[px];
        if (T * Ts < kTMin) {
            stop = j;
            break;
        }
        c0 = fmaf(T, r[1 * 256 + px], c0);
        c1 = fmaf(T, r[2 * 256 + px], c1);
        c2 = fmaf(T, r[3 * 256 + px], c2);
        D = fmaf(T, r[4 * 256 + px], D);
        T *= Ts;
        const int lj = reinterpret_cast<const int32_t*>(r)[5 * 256 + px];
        last = lj > 0 ? lj : last;
    }
    stop_row[px] = stop;
    if (stop < 0) {
        rgb[3 * p + 0] = fmaf(T, opt.bg[0], c0);
        rgb[3 * p + 1] = fmaf(T, opt.bg[1], c1);
        rgb[3 * p + 2] = fmaf(T, opt.bg[2], c2);
        alpha_out[p] = 1.0f - T;
    } else {
        rgb[3 * p + 0] = c0;
        rgb[3 * p + 1] = c1;
        rgb[3 * p + 2] = c2;
    }
    depth[p] = D;
    T_out[p] = T;
    last_out[p] = last;
}

// Pass 4, one workgroup per stored segment: the pixels that stop in this
// segment walk it again from their state before it, with the stop rule,
// T = T_start T_local and T_local recomputed as in pass 2 (so the pixel
// stops here, at the latest at the segment's last entry); they write their
// final outputs and the segment's state over the entries they composited
// (the state the backward folds).  (256, 7): 7 waves per SIMD, no spills.
__global__ __launch_bounds__(256, 7) void k_fwd_fix(const float4* __restrict__ rec,
                                                 const uint32_t* __restrict__ pair_vals,
                                                 const uint2* __restrict__ ranges,
                                                 const uint32_t* __restrict__ tile_order, ViewTable vt, OptK opt,
                                                 SegPlan plan, float* __restrict__ rgb, float* __restrict__ depth,
                                                 float* __restrict__ alpha_out, float* __restrict__ T_out,
                                                 int32_t* __restrict__ last_out) {
    __shared__ WaveStage stage[kWaves];
    const uint32_t b = blockIdx.x;
    if (b >= plan.state_off[plan.n_tiles]) return;
    const SegItem it = stored_seg(plan, b);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = order_tile(tile_order, vt, it.i);
    const PixelCoords pc = pixel_coords(vt, tile, wave, lane);
    const int px = pc.ly * kTile + pc.lx;
    bool alive = pc.inside && plan.stop_seg[(size_t)tile * 256 + px] == it.seg;
    const bool mine = alive;
    if (__ballot(alive) == 0) return;      // no pixel of the quadrant stops here
    WaveStage& st = stage[wave];
    const uint2 rg = ranges[tile];
    float Ts = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D0 = 0.0f;
    int last = 0;
    if (mine) {
        const int64_t p = pc.pix;
        Ts = T_out[p];
        C0 = rgb[3 * p + 0];
        C1 = rgb[3 * p + 1];
        C2 = rgb[3 * p + 2];
        D0 = depth[p];
        last = last_out[p];
    }
    const uint32_t lo = rg.x + (uint32_t)it.seg * kSegLen, hi = min(lo + (uint32_t)kSegLen, rg.y);
    float Tl = 1.0f, l0 = 0.0f, l1 = 0.0f, l2 = 0.0f, Dl = 0.0f;
    Gather cur = load_entry(rec, load_slot(pair_vals, lo + lane, hi));
    uint32_t s_next = load_slot(pair_vals, lo + kChunk + lane, hi);
    for (uint32_t j0 = lo; j0 < hi; j0 += kChunk) {
        if (__ballot(alive) == 0) break;
        const int n = stage_gathered(cur, (int)(j0 - rg.x) + lane + 1, pc, lane, st);
        cur = load_entry(rec, s_next);
        s_next = load_slot(pair_vals, j0 + 2 * kChunk + lane, hi);
        int last_k = -1;
        for (int k = 0; k < n; ++k) {
            const float4 a = st.g[k], bb = st.b[k], c = st.c[k];
            const Eval e = eval_entry(a, bb, pc.fpx, pc.fpy);
            const bool keep = alive && e.keep;
            const float Tln = Tl * (1.0f - e.alpha);
            const bool stop = keep && Ts * Tln < kTMin;
            const bool use = keep && !stop;
            const float w = use ? e.alpha * Tl : 0.0f;
            l0 = fmaf(c.x, w, l0);
            l1 = fmaf(c.y, w, l1);
            l2 = fmaf(c.z, w, l2);
            Dl = fmaf(bb.z, w, Dl);
            Tl = use ? Tln : Tl;
            last_k = use ? k : last_k;
            alive = alive && !stop;
        }
        if (last_k >= 0) last = st.ps[last_k].x;
        __builtin_amdgcn_wave_barrier();
    }
    if (!mine) return;
    const int64_t p = pc.pix;
    const float T = Ts * Tl;
    rgb[3 * p + 0] = fmaf(T, opt.bg[0], fmaf(Ts, l0, C0));
    rgb[3 * p + 1] = fmaf(T, opt.bg[1], fmaf(Ts, l1, C1));
    rgb[3 * p + 2] = fmaf(T, opt.bg[2], fmaf(Ts, l2, C2));
    depth[p] = fmaf(Ts, Dl, D0);
    alpha_out[p] = 1.0f - T;
    T_out[p] = T;
    last_out[p] = last;
    float* r = plan.state + (size_t)b * kSegFields * 256;
    r[0 * 256 + px] = Tl;
    r[1 * 256 + px] = l0;
    r[2 * 256 + px] = l1;
    r[3 * 256 + px] = l2;
    r[4 * 256 + px] = Dl;
}

// Persistent compositing: a fixed grid whose workgroups take tiles in launch
// order (longest lists first) from a counter until every tile is taken; the
// four waves composite the tile's quadrants, as in the one-tile-per-workgroup
// launch, so a tile's records are fetched into one compute unit's cache.  The
// next tile is taken while the current one composites.  A grid smaller than
// the device leaves compute units to work on other streams.
__global__ __launch_bounds__(256) void k_render_fwd_persistent(const float4* __restrict__ rec,
                                                               const uint32_t* __restrict__ pair_vals,
                                                               const uint2* __restrict__ ranges,
                                                               const uint32_t* __restrict__ tile_order, ViewTable vt,
                                                               OptK opt, float* __restrict__ rgb,
                                                               float* __restrict__ depth,
                                                               float* __restrict__ alpha_out,
                                                               float* __restrict__ T_out,
                                                               int32_t* __restrict__ last_out,
                                                               uint32_t* __restrict__ work) {
    __shared__ WaveStage stage[kWaves];
    __shared__ uint32_t s_item[2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t n_items = (uint32_t)vt.total_tiles;
    if (threadIdx.x == 0) s_item[0] = atomicAdd(work, 1u);
    __syncthreads();
    int k = 0;
    uint32_t item = s_item[0];
    // every wave of the workgroup reads the same item, so all leave together
    while (item < n_items) {
        if (threadIdx.x == 0) s_item[k ^ 1] = atomicAdd(work, 1u);
        render_fwd_quadrant(rec, pair_vals, ranges, vt, opt, order_tile(tile_order, vt, item), wave, lane,
                            stage[wave], rgb, depth, alpha_out, T_out, last_out);
        __syncthreads();     // the next item is in LDS; its slot is rewritten only after the next barrier
        k ^= 1;
        item = s_item[k];
    }
}

// Per pixel: the number of list entries compositing must evaluate -- those
// whose box contains the pixel centre, up to and including the one that
// stops the pixel.  The unit of work of compositing; measurement only.
__global__ __launch_bounds__(256) void k_render_count(const float4* __restrict__ rec,
                                                      const uint32_t* __restrict__ pair_vals,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ tile_order, ViewTable vt,
                                                      int32_t* __restrict__ n_eval) {
    __shared__ WaveStage stage[kWaves];
    __shared__ float2 sbox[kWaves][kChunk];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = launch_tile(tile_order, vt);
    const PixelCoords pc = pixel_coords(vt, tile, wave, lane);
    WaveStage& st = stage[wave];
    const uint2 rg = ranges[tile];
    float T = 1.0f;
    int count = 0, count_last = 0;
    bool alive = pc.inside;
    for (uint32_t j0 = rg.x; j0 < rg.y; j0 += kChunk) {
        if (__ballot(alive) == 0) break;
        const int n = stage_chunk(rec, pair_vals, rg.x, j0, rg.y, pc, lane, st);
        if (lane < n) {
            const float4 r3 = rec[4 * (size_t)(uint32_t)st.ps[lane].y + 3];
            sbox[wave][lane] = make_float2(r3.x, r3.y);
        }
        __builtin_amdgcn_wave_barrier();
        for (int k = 0; k < n; ++k) {
            const float4 a = st.g[k], b = st.b[k];
            const float2 h = sbox[wave][k];
            const bool covers = fabsf(pc.fpx - a.x) <= h.x && fabsf(pc.fpy - a.y) <= h.y;
            const Eval e = eval_entry(a, b, pc.fpx, pc.fpy);
            const float Tn = T * (1.0f - e.alpha);
            const bool keep = alive && e.keep;
            const bool stop = keep && Tn < kTMin;
            count += (alive && covers) ? 1 : 0;
            count_last = (keep && !stop) ? count : count_last;
            T = (keep && !stop) ? Tn : T;
            alive = alive && !stop;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (pc.inside) reinterpret_cast<int2*>(n_eval)[pc.pix] = make_int2(count, count_last);
}

__device__ __forceinline__ float row_total_lane15(float x) {
    // inclusive sums within each row of 16 lanes; lane 15 of the row ends with the row's total
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0.0f, x, 0x128, 0xf, 0xf, false);   // row_ror:8 (lane 15 + lane 7)
    // keeps the last add beside its DPP move (one v_add_f32_dpp) rather than
    // sunk into the caller's lane-15 branch; emits no instruction
    __asm__ volatile("" : "+v"(x));
    return x;
}

// Sums 12 per-lane values over the wave by halving exchanges: the lane
// halves swap six values (v_permlane32_swap) so that each half sums six
// fields over lane pairs, the rows swap three (v_permlane16_swap) so that
// each row of 16 sums three fields over 4 lanes, and DPP row shifts finish
// the three row sums.  Lane 16 r + 15 ends with the totals of fields
// 3r .. 3r + 2 in out[0..2] (30 VALU steps instead of 6 per field).
__device__ __forceinline__ void wave_sum12(const float v[12], float out[3]) {
    float a[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 6]), false,
                                                        false);
        // lanes 0-31: field j over (l, l + 32); lanes 32-63: field j + 6 over (l - 32, l)
        a[j] = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[j]), __float_as_uint(a[j + 3]), false,
                                                        false);
        // row r: field 3 r + j over the 4 lanes l, l +- 16, l +- 32 of its column
        out[j] = row_total_lane15(__uint_as_float(p[0]) + __uint_as_float(p[1]));
    }
}

// The same for fields 0 .. 9 (no AbsGS sums): five half swaps, three row
// swaps (the last with zeros).  Lane 16 r + 15 ends with fields b, b + 2
// and, for even r, b + 4 in out[0..2], where b = (r & 1) + 5 (r >> 1).
__device__ __forceinline__ void wave_sum10(const float v[10], float out[3]) {
    float a[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 5]), false,
                                                        false);
        // lanes 0-31: field j over (l, l + 32); lanes 32-63: field j + 5
        a[j] = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t x = __float_as_uint(a[2 * j]), y = j < 2 ? __float_as_uint(a[2 * j + 1]) : 0u;
        const auto p = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        out[j] = row_total_lane15(__uint_as_float(p[0]) + __uint_as_float(p[1]));
    }
}

constexpr int kG2 = GS_GRAD2D_FLOATS;   // per-slot 2D gradient fields

// Per-field factors applied once per entry, after the wave sum: the lanes
// sum dp (2 qa dx + qb dy), dp (qb dx + 2 qc dy), dp dx^2, dp dx dy, dp dy^2
// and the absolute values of the first two (dp = dL/d of the exponent in
// natural-log units), whose products with -ln2, -ln2, -1/2, -1, -1/2, ln2,
// ln2 are the gradients of the mean, of the conic (A, B, C) and the AbsGS
// sums.
__device__ __forceinline__ float grad2d_field_scale(int f) {
    return f < 2 ? -kLn2 : (f == 2 || f == 4) ? -0.5f : f == 3 ? -1.0f : f >= 10 ? kLn2 : 1.0f;
}

// Backward: each wave walks its quadrant's list back to front from the
// deepest `last` of its pixels, in chunks staged and culled as in the
// forward.  Per surviving entry the lanes' gradients are summed by
// wave_sum12 into a per-wave LDS row; after each chunk the wave adds the rows to the
// per-slot 2D gradient buffer with float atomics (zeros skipped).
// The colour and depth behind an entry enter the gradient only through
// their dot product with the pixel's upstream gradient, so the walk carries
// that one scalar, S = g_rgb . R_rgb + g_depth R_depth, instead of R itself.
template <bool kAbs>
__global__ __launch_bounds__(256) void k_render_bwd(const float4* __restrict__ rec,
                                                    const uint32_t* __restrict__ pair_vals,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ tile_order, ViewTable vt, OptK opt,
                                                    const float* __restrict__ T_final,
                                                    const int32_t* __restrict__ last_in,
                                                    const float* __restrict__ d_rgb, const float* __restrict__ d_depth,
                                                    const float* __restrict__ d_alpha, float* __restrict__ grad2d,
                                                    SegPlan plan) {
    __shared__ WaveStage stage[kWaves];
    // one row of reduced fields per staged entry of half a chunk (10 without
    // the AbsGS sums); the rows of a chunk's later half are flushed before
    // its earlier half reuses them, so seven workgroups share a compute
    // unit's LDS
    constexpr int kRow = kAbs ? kG2 : 10;
    constexpr int kRedRows = kChunk / 2;
    __shared__ float s_red[kWaves][kRedRows][kRow];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int tile, seg = 0, nseg = 1;
    uint32_t st0 = 0;
    if (plan.work_off) {
        // work item -> (launch position, segment)
        const uint32_t b = blockIdx.x;
        if (b >= plan.work_off[plan.n_tiles]) return;
        const uint32_t i = last_le(plan.work_off, plan.n_tiles, b);
        seg = (int)(b - plan.work_off[i]);
        nseg = (int)(plan.work_off[i + 1] - plan.work_off[i]);
        st0 = plan.state_off[i];
        tile = order_tile(tile_order, vt, i);
    } else {
        tile = launch_tile(tile_order, vt);
    }
    const PixelCoords pc = pixel_coords(vt, tile, wave, lane);
    WaveStage& st = stage[wave];
    const uint2 rg = ranges[tile];

    float T = 1.0f, gC0 = 0.0f, gC1 = 0.0f, gC2 = 0.0f, gD = 0.0f, gA = 0.0f;
    int last = 0;
    if (pc.inside) {
        const int64_t p = pc.pix;
        T = T_final[p];
        last = last_in[p];
        if (d_rgb) {
            gC0 = d_rgb[3 * p + 0];
            gC1 = d_rgb[3 * p + 1];
            gC2 = d_rgb[3 * p + 2];
        }
        if (d_depth) gD = d_depth[p];
        if (d_alpha) gA = d_alpha[p];
    }
    int maxlast = last;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, off, 64));

    // R = remaining colour behind the entry divided by T after it (starts at
    // bg); the walk keeps S = g . R
    float S = fmaf(gC0, opt.bg[0], fmaf(gC1, opt.bg[1], gC2 * opt.bg[2])), Q = 1.0f;

    // A segmented list: this workgroup walks segment `seg` (positions
    // (seg S, (seg + 1) S]); the state behind it comes from folding the later
    // segments' transmittance and local colour, written by k_seg_prepass:
    // R <- C_j + T_j R (so S <- g . C_j + T_j S), T <- T / T_j, Q <- Q T_j
    // (segments starting at or after the pixel's last composited entry are
    // the identity).
    int lo = 0, hi = maxlast;
    if (nseg > 1) {
        const int px = pc.ly * kTile + pc.lx;
        for (int j = nseg - 1; j > seg; --j) {
            if (j * kSegLen >= last) continue;
            const float* sj = plan.state + (size_t)(st0 + (uint32_t)(j - 1)) * kSegFields * 256;
            const float Ts = sj[0 * 256 + px];
            const float gcs = fmaf(gC0, sj[1 * 256 + px],
                                   fmaf(gC1, sj[2 * 256 + px], fmaf(gC2, sj[3 * 256 + px], gD * sj[4 * 256 + px])));
            S = fmaf(Ts, S, gcs);
            T = T / Ts;
            Q = Q * Ts;
        }
        lo = seg * kSegLen;
        hi = min((seg + 1) * kSegLen, maxlast);
    }

    // chunk [b_end - 64, b_end) of positions, clipped at lo, walked from the
    // back; lane l of a chunk gathers position b_start + l
    auto chunk_slot = [&](int b_end_) {
        const int b_start_ = max(lo, b_end_ - kChunk);
        return b_end_ > lo ? load_slot(pair_vals, rg.x + (uint32_t)(b_start_ + lane), rg.x + (uint32_t)b_end_) : kNoSlot;
    };
    // adds the sums of staged entries [k0, k1) (one half of the staged
    // chunk, rows k mod kRedRows) to grad2d
    constexpr int kFields = kAbs ? kG2 : 10;
    auto flush = [&](int k0, int k1) {
        for (int i = lane; i < (k1 - k0) * kFields; i += 64) {
            const int j = i / kFields, f = i - j * kFields, k = k0 + j;
            const float sum = s_red[wave][k & (kRedRows - 1)][f];
            if (sum != 0.0f)
                atomicAdd(&grad2d[(size_t)(uint32_t)st.ps[k].y * kG2 + f], sum * grad2d_field_scale(f));
        }
        __builtin_amdgcn_wave_barrier();
    };
    Gather cur = load_entry(rec, chunk_slot(hi));
    uint32_t s_next = chunk_slot(hi - kChunk);
    int n_prev = 0;
    for (int b_end = hi; b_end > lo; b_end -= kChunk) {
        const int b_start = max(lo, b_end - kChunk);
        // Wait for this chunk's records here, then issue the previous
        // chunk's atomics: loads and atomics share one in-order counter, so
        // atomics issued before the wait would be waited for as well.
        __asm__ volatile("" ::"v"(cur.r0.x), "v"(cur.r1.x), "v"(cur.r2.x), "v"(cur.r3.x), "v"(s_next));
        flush(0, min(n_prev, kRedRows));
        const int n = stage_gathered(cur, b_start + lane + 1, pc, lane, st);
        n_prev = n;
        cur = load_entry(rec, s_next);
        s_next = chunk_slot(b_end - 2 * kChunk);
        for (int k = n - 1; k >= 0; --k) {
            const float4 a = st.g[k], b = st.b[k], c = st.c[k];
            // whole-record reads at the entry's one LDS address (b.w and c.w
            // are used only under the ballot below); emits no instruction
            __asm__ volatile("" ::"v"(b.w), "v"(c.w));
            const int pos = st.ps[k].x;       // 1-based
            const Eval e = eval_entry(a, b, pc.fpx, pc.fpy);
            const bool con = pos <= last && e.keep;
            // an entry the pixel did not composite takes alpha = 0, which
            // leaves S and Q unchanged exactly (x 1, + 0)
            const float al = con ? e.alpha : 0.0f;
            const float one_m = 1.0f - al;
            const float Ti = T * __builtin_amdgcn_rcpf(one_m);
            const float gc = fmaf(gC0, c.x, fmaf(gC1, c.y, fmaf(gC2, c.z, gD * b.z)));   // g . (colour, depth)
            const float dal = Ti * fmaf(gA, Q, gc - S);
            const float w = al * Ti;
            float g[kG2];
            g[6] = gC0 * w;
            g[7] = gC1 * w;
            g[8] = gC2 * w;
            g[9] = gD * w;
            const float dal_u = (con && e.raw < kAlphaMax) ? dal : 0.0f;
            g[5] = dal_u * e.G;
            const float dp = dal_u * al;               // dL/d power (natural-log units)
            const float dpx = dp * e.dx, dpy = dp * e.dy;
            g[0] = fmaf(c.w, dpx, a.w * dpy);         // dp (2 qa dx + qb dy)
            g[1] = fmaf(a.w, dpx, b.w * dpy);         // dp (qb dx + 2 qc dy)
            g[2] = dpx * e.dx;
            g[3] = dpx * e.dy;
            g[4] = dpy * e.dy;
            if (kAbs) {
                g[10] = fabsf(g[0]);
                g[11] = fabsf(g[1]);
            }
            S = fmaf(S, one_m, gc * al);
            Q *= one_m;
            T = con ? Ti : T;
            if (kAbs) {
                // lane 16 r + 15 writes fields 3 r .. 3 r + 2 of the entry's row
                float* row = &s_red[wave][k & (kRedRows - 1)][3 * (lane >> 4)];
                if (__ballot(con)) {
                    float tot[3];
                    wave_sum12(g, tot);
                    if ((lane & 15) == 15) {
                        row[0] = tot[0];
                        row[1] = tot[1];
                        row[2] = tot[2];
                    }
                } else if ((lane & 15) == 15) {
                    row[0] = row[1] = row[2] = 0.0f;
                }
            } else {
                // lane 16 r + 15 writes its fields of the entry's row
                const int r = lane >> 4;
                float* row = &s_red[wave][k & (kRedRows - 1)][(r & 1) + 5 * (r >> 1)];
                float tot[3] = {0.0f, 0.0f, 0.0f};
                if (__ballot(con)) wave_sum10(g, tot);
                if ((lane & 15) == 15) {
                    row[0] = tot[0];
                    row[2] = tot[1];
                    if (!(r & 1)) row[4] = tot[2];
                }
            }
            // the later half's rows go out before the earlier half reuses them
            if (k == kRedRows) flush(kRedRows, n);
        }
        __builtin_amdgcn_wave_barrier();
    }
    flush(0, min(n_prev, kRedRows));
}

// exclusive scan of v over the 1024 threads of the workgroup; *total gets the sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
        const uint32_t t = s_wave[w];
        before += w < wave ? t : 0u;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// One workgroup: segments per tile in launch order (ceil(L / kSegLen) for a
// list of L > kSegLen positions, else 1) and the stored states (segments
// 1 .. n - 1); exclusive prefix sums into work_off / state_off.  When the
// states would exceed `capacity`, every tile keeps a single segment.  Thread
// t takes the consecutive positions [t k, t k + k), so the prefix sums need
// one workgroup scan of the threads' totals, not one per 1024 tiles; the
// counts of up to kPlanCache tiles stay in LDS between the two passes.
constexpr uint32_t kPlanCache = 32640;
constexpr int kPlanBatch = 8;
__global__ __launch_bounds__(1024) void k_seg_plan(const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ tile_order, ViewTable vt,
                                                   uint32_t capacity, uint32_t* __restrict__ work_off,
                                                   uint32_t* __restrict__ state_off) {
    __shared__ uint32_t s_wave[16];
    __shared__ uint16_t s_nseg[kPlanCache];
    const uint32_t n_tiles = (uint32_t)vt.total_tiles;
    // segment counts of the launch positions [ib, min(ib + kPlanBatch, end))
    auto nseg_batch = [&](uint32_t ib, uint32_t end, uint32_t* c) {
        int t[kPlanBatch];
#pragma unroll
        for (int u = 0; u < kPlanBatch; ++u) t[u] = ib + u < end ? order_tile(tile_order, vt, ib + u) : -1;
        uint2 r[kPlanBatch];
#pragma unroll
        for (int u = 0; u < kPlanBatch; ++u) r[u] = t[u] >= 0 ? ranges[t[u]] : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < kPlanBatch; ++u) {
            const uint32_t L = r[u].y - r[u].x;
            c[u] = L > (uint32_t)kSegLen ? (L + kSegLen - 1) / kSegLen : 1u;
        }
    };
    const uint32_t k = (n_tiles + 1023) / 1024;
    const uint32_t i0 = threadIdx.x * k, i1 = min(i0 + k, n_tiles);
    // pass 1: the thread's segment total (cached counts below 2^16).  The
    // positions are read kPlanBatch at a time, all loads first, so a thread
    // waits for one round of gathers per batch instead of one per position
    uint32_t mine = 0, big = 0;
    for (uint32_t ib = i0; ib < i1; ib += kPlanBatch) {
        uint32_t c[kPlanBatch];
        nseg_batch(ib, i1, c);
#pragma unroll
        for (int u = 0; u < kPlanBatch; ++u) {
            const uint32_t i = ib + u;
            if (i >= i1) break;
            mine += c[u];
            if (i < kPlanCache) s_nseg[i] = (uint16_t)c[u];
            big |= c[u] > 0xFFFFu ? 1u : 0u;
        }
    }
    // the threads' prefix and the total (do the states fit?), and whether
    // any count was too large for the cache
    uint32_t total_seg = 0, total_big = 0;
    const uint32_t before_seg = block_excl_scan(mine, s_wave, &total_seg);
    (void)block_excl_scan(big, s_wave, &total_big);      // its barriers also publish s_nseg
    const uint32_t total_need = total_seg - n_tiles;
    const bool on = total_need <= capacity;
    const bool cached = total_big == 0;
    // pass 2: each position's offsets from the thread's exclusive prefix
    uint32_t w = on ? before_seg : i0, st = on ? before_seg - i0 : 0u;
    for (uint32_t ib = i0; ib < i1; ib += kPlanBatch) {
        uint32_t c[kPlanBatch];
        if (on && !(cached && ib + kPlanBatch <= kPlanCache)) nseg_batch(ib, i1, c);
#pragma unroll
        for (int u = 0; u < kPlanBatch; ++u) {
            const uint32_t i = ib + u;
            if (i >= i1) break;
            const uint32_t ci = on ? (cached && i < kPlanCache ? (uint32_t)s_nseg[i] : c[u]) : 1u;
            work_off[i] = w;
            state_off[i] = st;
            w += ci;
            st += ci - 1u;
        }
    }
    if (threadIdx.x == 1023) {
        work_off[n_tiles] = on ? total_seg : n_tiles;
        state_off[n_tiles] = on ? total_need : 0u;
    }
}

// State of one stored segment (tile at launch position i, segment j >= 1):
// per pixel, front to back over the segment's composited entries (position
// <= last and not skipped), T_seg = prod (1 - alpha) and the colour and
// depth sums with T restarted at 1: C_seg = sum c alpha T_local.  The
// alpha values are the forward's and the backward's bit for bit.
__global__ __launch_bounds__(256) void k_seg_prepass(const float4* __restrict__ rec,
                                                     const uint32_t* __restrict__ pair_vals,
                                                     const uint2* __restrict__ ranges,
                                                     const uint32_t* __restrict__ tile_order, ViewTable vt,
                                                     const int32_t* __restrict__ last_in, SegPlan plan) {
    __shared__ WaveStage stage[kWaves];
    const uint32_t b = blockIdx.x;
    if (b >= plan.state_off[plan.n_tiles]) return;
    const uint32_t i = last_le(plan.state_off, plan.n_tiles, b);
    const int j = (int)(b - plan.state_off[i]) + 1;
    const int tile = order_tile(tile_order, vt, i);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const PixelCoords pc = pixel_coords(vt, tile, wave, lane);
    WaveStage& st = stage[wave];
    const uint2 rg = ranges[tile];
    const int last = pc.inside ? last_in[pc.pix] : 0;
    int maxlast = last;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, off, 64));
    const int lo = j * kSegLen, hi = min((j + 1) * kSegLen, maxlast);
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, D = 0.0f;
    for (int b0 = lo; b0 < hi; b0 += kChunk) {
        const Gather e = load_entry(rec, load_slot(pair_vals, rg.x + (uint32_t)(b0 + lane), rg.x + (uint32_t)hi));
        const int n = stage_gathered(e, b0 + lane + 1, pc, lane, st);
        for (int k = 0; k < n; ++k) {
            const float4 a = st.g[k], bb = st.b[k], c = st.c[k];
            const Eval ev = eval_entry(a, bb, pc.fpx, pc.fpy);
            const bool con = st.ps[k].x <= last && ev.keep;
            const float w = con ? ev.alpha * T : 0.0f;
            c0 = fmaf(c.x, w, c0);
            c1 = fmaf(c.y, w, c1);
            c2 = fmaf(c.z, w, c2);
            D = fmaf(bb.z, w, D);
            T = con ? T * (1.0f - ev.alpha) : T;
        }
        __builtin_amdgcn_wave_barrier();
    }
    float* out = plan.state + (size_t)b * kSegFields * 256;
    const int px = pc.ly * kTile + pc.lx;
    out[0 * 256 + px] = T;
    out[1 * 256 + px] = c0;
    out[2 * 256 + px] = c1;
    out[3 * 256 + px] = c2;
    out[4 * 256 + px] = D;
}

// 2D-gradient rows of the slots that some tile lists (tiles > 0): the only
// rows the compositing backward accumulates into and the only ones read
__global__ __launch_bounds__(256) void k_zero_seen_rows(const uint32_t* __restrict__ tiles, float4* __restrict__ grad2d,
                                                        int64_t n_slots) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_slots || tiles[i] == 0) return;
    const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    grad2d[3 * i + 0] = z;
    grad2d[3 * i + 1] = z;
    grad2d[3 * i + 2] = z;
}

}  // namespace

hipError_t launch_render_fwd(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                             const ViewTable& vt, const OptK& opt, float* rgb, float* depth, float* alpha,
                             float* T_final, int32_t* last, hipStream_t s, int persistent_ctas, uint32_t* work,
                             const SegPlan* plan) {
    if (vt.total_tiles <= 0) return hipSuccess;
    const hipEvent_t timed_ = timer_begin(GS_KERNEL_RENDER_FWD, s);
    if (persistent_ctas > 0 && work) {
        hipError_t e = fill_u32(work, 0u, 1, s);
        if (e != hipSuccess) return e;
        const int grid = persistent_ctas < vt.total_tiles ? persistent_ctas : vt.total_tiles;
        hipLaunchKernelGGL(k_render_fwd_persistent, dim3(grid), dim3(256), 0, s, proj.rec, pair_vals, ranges,
                           proj.tile_order, vt, opt, rgb, depth, alpha, T_final, last, work);
    } else {
        const SegPlan none{nullptr, nullptr, nullptr, (uint32_t)vt.total_tiles, nullptr, 0u};
        hipLaunchKernelGGL(k_render_fwd, dim3(vt.total_tiles), dim3(256), 0, s, proj.rec, pair_vals, ranges,
                           proj.tile_order, vt, opt, rgb, depth, alpha, T_final, last, plan ? *plan : none);
        if (plan && plan->capacity) {
            // the later segments of the planned lists, the fold, and the
            // re-walk of the segments pixels stop in
            hipLaunchKernelGGL(k_fwd_segments, dim3(plan->capacity), dim3(256), 0, s, proj.rec, pair_vals, ranges,
                               proj.tile_order, vt, *plan);
            hipLaunchKernelGGL(k_fwd_combine, dim3(vt.total_tiles), dim3(256), 0, s, proj.tile_order, vt, opt, *plan,
                               rgb, depth, alpha, T_final, last);
            hipLaunchKernelGGL(k_fwd_fix, dim3(plan->capacity), dim3(256), 0, s, proj.rec, pair_vals, ranges,
                               proj.tile_order, vt, opt, *plan, rgb, depth, alpha, T_final, last);
        }
    }
    timer_end(timed_, s);
    return hipGetLastError();
}

hipError_t launch_render_count(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                               const ViewTable& vt, int32_t* n_eval, hipStream_t s) {
    if (vt.total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_render_count, dim3(vt.total_tiles), dim3(256), 0, s, proj.rec, pair_vals, ranges,
                       proj.tile_order, vt, n_eval);
    return hipGetLastError();
}

hipError_t launch_seg_plan(const Projected& proj, const uint2* ranges, const ViewTable& vt, uint32_t capacity,
                           const SegPlan& plan, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_plan, dim3(1), dim3(1024), 0, s, ranges, proj.tile_order, vt, capacity, plan.work_off,
                       plan.state_off);
    return hipGetLastError();
}

hipError_t launch_seg_prepare(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                              const ViewTable& vt, const int32_t* last, uint32_t capacity, const SegPlan& plan,
                              hipStream_t s) {
    hipError_t e = launch_seg_plan(proj, ranges, vt, capacity, plan, s);
    if (e != hipSuccess) return e;
    if (capacity)
        hipLaunchKernelGGL(k_seg_prepass, dim3(capacity), dim3(256), 0, s, proj.rec, pair_vals, ranges, proj.tile_order,
                           vt, last, plan);
    return hipGetLastError();
}

hipError_t launch_render_bwd(const Projected& proj, const uint32_t* pair_vals, const uint2* ranges,
                             const ViewTable& vt, const OptK& opt, const float* T_final, const int32_t* last,
                             const float* d_rgb, const float* d_depth, const float* d_alpha, float* grad2d,
                             const SegPlan& plan, uint32_t capacity, bool abs_sums, hipStream_t s) {
    // with a plan, blocks beyond the planned work items exit at once
    const unsigned blocks = (unsigned)vt.total_tiles + (plan.work_off ? capacity : 0u);
    const hipEvent_t timed_ = timer_begin(GS_KERNEL_RENDER_BWD, s);
    if (abs_sums)
        hipLaunchKernelGGL(k_render_bwd<true>, dim3(blocks), dim3(256), 0, s, proj.rec, pair_vals, ranges,
                           proj.tile_order, vt, opt, T_final, last, d_rgb, d_depth, d_alpha, grad2d, plan);
    else
        hipLaunchKernelGGL(k_render_bwd<false>, dim3(blocks), dim3(256), 0, s, proj.rec, pair_vals, ranges,
                           proj.tile_order, vt, opt, T_final, last, d_rgb, d_depth, d_alpha, grad2d, plan);
    timer_end(timed_, s);
    return hipGetLastError();
}

hipError_t zero_seen_grad2d(const uint32_t* tiles, float* grad2d, int64_t n_slots, hipStream_t s) {
    const unsigned blocks = (unsigned)((n_slots + 255) / 256);
    hipLaunchKernelGGL(k_zero_seen_rows, dim3(blocks), dim3(256), 0, s, tiles, reinterpret_cast<float4*>(grad2d),
                       n_slots);
    return hipGetLastError();
}

}  // namespace gs
