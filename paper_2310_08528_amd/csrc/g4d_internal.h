// Internal definitions shared by the HIP translation units of libg4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "../../include/g4d.h"

namespace g4d {

constexpr int kTile = G4D_TILE;              // 16x16 pixel tiles
constexpr int kTilePixels = kTile * kTile;   // one blend block per tile

// Radix-sort tiling: 256 threads x kSortItems keys per block.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // 2048 keys per block (instances)
constexpr int kSortItemsN = 4;
constexpr int kSortTileN = kSortThreads * kSortItemsN; // 1024 keys per block (per-Gaussian depth)
constexpr int kScanTile = 256 * 16;                    // 4096 values per scan block

// Lookback status words: flag in the top two bits, value in the low 30.
constexpr uint32_t kFlagShift = 30;
constexpr uint32_t kValueMask = (1u << kFlagShift) - 1u;
constexpr uint32_t kFlagAggregate = 1u;
constexpr uint32_t kFlagInclusive = 2u;
constexpr uint32_t kSpinLimit = 1u << 22;    // bounded wait: gives up and flags an error

// Device status block at the start of the workspace.
struct DevStatus {
    unsigned long long k_total;      // instances the frame needs
    uint32_t k_used;                 // min(k_total, capacity)
    uint32_t overflow;
    uint32_t sort_error;
    uint32_t visible;
    uint32_t tiles;
    uint32_t passes;
    uint32_t tile_counter[16];       // onesweep tile tickets, one per sort pass / scan
    uint32_t pack_bits;              // instances packed as (tile << pack_bits) | index; 0: two arrays
    uint32_t tracked;                // the last blend counted its work (n_contrib / final_T requested)
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline int ceil_log2(uint32_t x) {
    int b = 0;
    while ((1u << b) < x) ++b;
    return b;
}

// Byte offsets of every array in a render workspace.  The first `zero_bytes`
// bytes are cleared at the start of each render.
struct WsLayout {
    int32_t n_max, w_max, h_max;
    int64_t cap;
    int32_t tiles_max;
    int32_t nblk_n;      // sort blocks over n
    int32_t nblk_k;      // sort blocks over capacity
    int32_t nscan;       // scan blocks over n
    size_t status, depth_hist, lb_depth, lb_scan, ranges;
    size_t tgrid;        // tile-count difference grid [tiles_y + 1][tiles_x + 1] (int32), cleared per render
    size_t zero_bytes;
    size_t cam;
    size_t recA, recB, recC, rect, touched, dgid, dk0, dk1, dv0, dv1, offsets, tk0, tk1, tv0, tv1;
    size_t tcnt, tdtot;  // instance sort: per-pass digit counts [256][nblk_k] and digit totals [256]
    size_t order;        // blend order of the tiles (longest list first): (tile, start, end, 0)
    size_t evals;        // per tile: (pixel, Gaussian) pairs the blend evaluated (u64)
    size_t comp;         // per tile: kept (pixel, Gaussian) pairs the blend composited (u64)
    size_t grad2d;       // render backward: per Gaussian dL/d(u, v, conic A B C, colour r g b, opacity), [9][n]
    size_t total;
};

inline bool make_layout(int32_t n, int32_t w, int32_t h, int64_t cap, WsLayout *L) {
    if (n < 0 || n > (1 << 26) || w < 1 || h < 1 || w > 4096 || h > 4096 || cap < 1 ||
        cap >= (int64_t(1) << 30))
        return false;
    L->n_max = n; L->w_max = w; L->h_max = h; L->cap = cap;
    int tx = (w + kTile - 1) / kTile, ty = (h + kTile - 1) / kTile;
    L->tiles_max = tx * ty;
    int32_t nn = n > 0 ? n : 1;
    L->nblk_n = (nn + kSortTileN - 1) / kSortTileN;
    L->nblk_k = (int32_t)((cap + kSortTile - 1) / kSortTile);
    L->nscan = (nn + kScanTile - 1) / kScanTile;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
    L->status = take(sizeof(DevStatus));
    L->depth_hist = take(4 * 256 * 4);
    L->lb_depth = take((size_t)4 * L->nblk_n * 256 * 4);
    L->lb_scan = take((size_t)L->nscan * 8);
    L->ranges = take((size_t)L->tiles_max * 8);
    L->tgrid = take((size_t)(tx + 1) * (ty + 1) * 4);
    L->zero_bytes = o;
    L->cam = take(256);
    L->recA = take((size_t)nn * 16);
    L->recB = take((size_t)nn * 16);
    L->recC = take((size_t)nn * 16);
    L->rect = take((size_t)nn * 8);
    L->touched = take((size_t)nn * 4);
    L->dgid = take((size_t)nn * 4);
    L->dk0 = take((size_t)nn * 4);
    L->dk1 = take((size_t)nn * 4);
    L->dv0 = take((size_t)nn * 4);
    L->dv1 = take((size_t)nn * 4);
    L->offsets = take((size_t)nn * 8);
    L->tk0 = take((size_t)cap * 4);
    L->tk1 = take((size_t)cap * 4);
    L->tv0 = take((size_t)cap * 4);
    L->tv1 = take((size_t)cap * 4);
    L->tcnt = take((size_t)2 * 256 * L->nblk_k * 4);
    L->tdtot = take((size_t)2 * 256 * 4);
    L->order = take((size_t)L->tiles_max * 16);
    L->evals = take((size_t)L->tiles_max * 8);
    L->comp = take((size_t)L->tiles_max * 8);
    L->grad2d = take((size_t)nn * 9 * 4);
    L->total = o;
    return true;
}

// Sort-pass plan for the tile ids of a frame with `tiles` tiles: digit
// widths of at most 8 bits, balanced over the passes.
struct TilePassPlan {
    int passes;
    int shift[2];
    int bits[2];
};

inline TilePassPlan tile_pass_plan(int tiles) {
    TilePassPlan p{};
    int b = ceil_log2((uint32_t)(tiles > 1 ? tiles : 2));
    if (b <= 8) {
        p.passes = 1; p.shift[0] = 0; p.bits[0] = b;
    } else {
        p.passes = 2;
        p.bits[0] = (b + 1) / 2; p.shift[0] = 0;
        p.bits[1] = b - p.bits[0]; p.shift[1] = p.bits[0];
    }
    return p;
}

// Host-side error plumbing.
void set_hip_error(hipError_t e);

// Entry points shared between translation units.
g4d_status render(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws, float *image,
                  float *final_T, int32_t *n_contrib, hipStream_t s);
g4d_status read_status(const g4d_workspace *ws, g4d_device_status *out, hipStream_t s);
g4d_status spatial_order(const g4d_gaussians *G, const float bmin[3], const float bmax[3],
                         const g4d_workspace *ws, uint32_t *order, hipStream_t s);
g4d_status deform_batched(const g4d_deform_job *jobs, int n_jobs, hipStream_t s);
g4d_status deform_backward(const g4d_gaussians *G, const g4d_planes *P, const g4d_mlp *M, float t,
                           const g4d_splats_grad *gout, const g4d_deform_grad *d, hipStream_t s);
g4d_status render_backward(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws,
                           const float *final_T, const int32_t *n_contrib, const float *grad_image,
                           const g4d_splats_grad *out, hipStream_t s);
g4d_status graph_find_camera_node(hipGraph_t g, hipGraphNode_t *out);
g4d_status graph_set_frame(hipGraphExec_t exec, hipGraphNode_t node, const g4d_workspace *ws,
                           const g4d_camera *C, float *image, float *final_T, int32_t *n_contrib);
// Byte offset of the device status block inside a workspace.
size_t status_offset(const g4d_workspace *ws);

// Stage events of the calling thread (null when off).
constexpr int kStageEvents = 9;
hipEvent_t stage_event(int i);

}  // namespace g4d

#define G4D_HIP_CHECK(expr)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) {                               \
            g4d::set_hip_error(_e);                           \
            return G4D_EHIP;                                  \
        }                                                     \
    } while (0)

namespace g4d {

// Raises a kernel's dynamic-LDS limit to `bytes` once per device (the
// attribute is held per device); `done` holds one bit per device id and may
// be shared by concurrent callers.
inline g4d_status ensure_max_lds(const void *fn, std::atomic<uint64_t> &done, int bytes) {
    int dev = 0;
    G4D_HIP_CHECK(hipGetDevice(&dev));
    const uint64_t bit = (dev >= 0 && dev < 64) ? (1ull << dev) : 0ull;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return G4D_OK;
    G4D_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    if (bit) done.fetch_or(bit, std::memory_order_release);
    return G4D_OK;
}

}  // namespace g4d
