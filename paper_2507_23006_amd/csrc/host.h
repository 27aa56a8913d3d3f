// Host-side helpers shared by the C ABI translation units: error reporting,
// argument checks, per-view constant tables, workspace carving and the
// binning launch sequence.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gs.h"
#include "gs_internal.h"

namespace gs {
namespace host {

// sets the calling thread's error message and returns `code`
int fail(int code, const char* fmt, ...);
const char* last_error();

#define GS_HIP(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return ::gs::host::fail(GS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define GS_REQUIRE(cond, ...)                                               \
    do {                                                                    \
        if (!(cond)) return ::gs::host::fail(GS_ERR_INVALID_ARG, __VA_ARGS__); \
    } while (0)

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// carves aligned regions out of a workspace; with base == nullptr it only
// measures
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off = align_up(off + count * sizeof(T));
        return p;
    }
};

int build_views(const gs_camera* cams, int32_t n_views, ViewTable* vt);
int build_opt(const gs_options* o, OptK* k);

// segment area of the segmented compositing: work_off [T + 1] | state_off
// [T + 1] | stop_seg [T][256] | states [capacity][kSegFields][256]; the
// fixed part's bytes, and the plan over an area (NULL or smaller than the
// fixed part: no segments)
size_t seg_fixed_bytes(int64_t n_tiles);
void seg_layout(void* base, size_t bytes, int64_t n_tiles, SegPlan* plan, uint32_t* capacity);

// workspace bytes of bin_sort_slots
size_t bin_workspace_bytes(int64_t n_slots, int64_t pair_capacity);

// depth sort of n_slots projected slots, pair emission, tile sort and tile
// ranges for the views of vt; asynchronous: the pair count is written to
// the device int64 *n_pairs_dev, and a count above pair_capacity leaves
// every tile range empty
int bin_sort_slots(const Projected& pr, const ViewTable& vt, int64_t n_slots, int64_t pair_capacity,
                   uint32_t* pair_vals, uint32_t* tile_ranges, int64_t* n_pairs_dev, void* ws, size_t ws_bytes,
                   hipStream_t s);

}  // namespace host
}  // namespace gs
