// g4d_render_noalloc: the render of g4d_render with its workspace held in a
// fixed device array of this library instead of a caller buffer, for callers
// that cannot allocate device memory (code under graph capture, serving
// loops that forbid allocation, harnesses that disallow it).
//
// The array `scratch` is a file-scope __device__ object: every GPU the
// library runs on holds its own copy, for the life of the process.  Its name
// in host code is only a host-side stand-in, so the device address is looked
// up once per device with hipGetSymbolAddress and that pointer is what the
// kernels receive.  Every call on a GPU shares that GPU's copy: calls that
// overlap on one device (two streams, two threads) race on it.  The render's
// first kernel clears the counters, histograms, look-back state and ranges
// it needs at zero, so a call does not depend on what the previous one left.
#include "g4d_internal.h"

#include <mutex>

static __device__ __align__(256) unsigned char scratch[G4D_NOALLOC_SCRATCH_BYTES];

namespace g4d {
namespace {

constexpr size_t kScratchBytes = size_t(G4D_NOALLOC_SCRATCH_BYTES);
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up on the first
// call on that device (with the device current) and kept.
g4d_status scratch_ptr(void **out) {
    int dev = 0;
    G4D_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return G4D_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        G4D_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) return G4D_EDEVICE;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return G4D_OK;
}

// Largest instance capacity whose workspace layout for (n, w, h) fits the
// scratch array; 0 if not even one instance fits.  The layout size grows
// with the capacity, so a binary search finds it.
int64_t capacity_in_scratch(int32_t n, int32_t w, int32_t h) {
    WsLayout L;
    if (!make_layout(n, w, h, 1, &L) || L.total > kScratchBytes) return 0;
    int64_t lo = 1, hi = (int64_t(1) << 30) - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (make_layout(n, w, h, mid, &L) && L.total <= kScratchBytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

}  // namespace
}  // namespace g4d

extern "C" g4d_status g4d_render_noalloc(const g4d_splats *G, const g4d_camera *C, float *image, float *final_T,
                                         int32_t *n_contrib, g4d_device_status *status, void *stream) {
    using namespace g4d;
    if (!G || !C || !image) return G4D_EINVAL;
    if (G->n < 0 || C->width < 1 || C->height < 1 || C->width > 4096 || C->height > 4096) return G4D_EINVAL;
    // sizes beyond what the fixed array holds are refused before any HIP call
    const int64_t cap = capacity_in_scratch(std::max(G->n, 1), C->width, C->height);
    if (cap < 1) return G4D_ENOMEM;
    void *p = nullptr;
    if (g4d_status e = scratch_ptr(&p)) return e;
    g4d_workspace ws{};
    ws.ptr = p;
    ws.bytes = kScratchBytes;
    ws.n_max = std::max(G->n, 1);
    ws.width_max = C->width;
    ws.height_max = C->height;
    ws.instance_capacity = cap;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (g4d_status e = render(G, C, &ws, image, final_T, n_contrib, s)) return e;
    if (!status) return G4D_OK;
    // outcome of this frame: the status block only (no per-tile counts, which
    // would need a host buffer sized by the frame)
    DevStatus h{};
    G4D_HIP_CHECK(hipMemcpyAsync(&h, static_cast<char *>(p) + status_offset(&ws), sizeof(h), hipMemcpyDeviceToHost,
                                 s));
    G4D_HIP_CHECK(hipStreamSynchronize(s));
    status->instances = (int64_t)h.k_total;
    status->overflow = (int32_t)h.overflow;
    status->sort_error = (int32_t)h.sort_error;
    status->visible = (int32_t)h.visible;
    status->tiles = (int32_t)h.tiles;
    status->blend_evals = -1;
    status->blend_composited = -1;
    if (h.overflow) return G4D_ECAPACITY;
    if (h.sort_error) return G4D_EDEVICE;
    return G4D_OK;
}
