// C ABI entry points of libg4d that are not defined next to their kernels:
// render wrappers, status/error plumbing and version.
#include "g4d_internal.h"

namespace g4d {
g4d_status render_export(const g4d_workspace *ws, int32_t kind, int32_t n, int64_t k, void *dst, size_t bytes,
                         hipStream_t s);

namespace {
thread_local int32_t g_last_hip_error = 0;
thread_local hipEvent_t g_stage_events[kStageEvents] = {};
thread_local bool g_stage_on = false;
}

void set_hip_error(hipError_t e) { g_last_hip_error = (int32_t)e; }

hipEvent_t stage_event(int i) { return g_stage_on && i >= 0 && i < kStageEvents ? g_stage_events[i] : nullptr; }

}  // namespace g4d

extern "C" size_t g4d_render_workspace_bytes(int32_t n, int32_t width, int32_t height, int64_t instance_capacity) {
    g4d::WsLayout L;
    if (!g4d::make_layout(n, width, height, instance_capacity, &L)) return 0;
    return L.total;
}

extern "C" g4d_status g4d_render(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws, float *image,
                                 float *final_T, int32_t *n_contrib, void *stream) {
    return g4d::render(G, C, ws, image, final_T, n_contrib, reinterpret_cast<hipStream_t>(stream));
}

extern "C" g4d_status g4d_spatial_order(const g4d_gaussians *G, const float bmin[3], const float bmax[3],
                                        const g4d_workspace *ws, uint32_t *order, void *stream) {
    return g4d::spatial_order(G, bmin, bmax, ws, order, reinterpret_cast<hipStream_t>(stream));
}

extern "C" g4d_status g4d_read_status(const g4d_workspace *ws, g4d_device_status *out, void *stream) {
    return g4d::read_status(ws, out, reinterpret_cast<hipStream_t>(stream));
}

extern "C" g4d_status g4d_render_export(const g4d_workspace *ws, int32_t kind, int32_t n, int64_t k, void *dst,
                                        size_t dst_bytes, void *stream) {
    return g4d::render_export(ws, kind, n, k, dst, dst_bytes, reinterpret_cast<hipStream_t>(stream));
}

extern "C" const char *g4d_status_string(int32_t status) {
    switch (status) {
        case G4D_OK: return "ok";
        case G4D_EINVAL: return "invalid argument";
        case G4D_EUNSUPPORTED: return "unsupported shape";
        case G4D_ECAPACITY: return "instance capacity exceeded";
        case G4D_EHIP: return "HIP runtime error";
        case G4D_EBUSY: return "busy";
        case G4D_ENOMEM: return "request exceeds the memory budget or the fixed scratch array";
        case G4D_ENOTFOUND: return "not found";
        case G4D_EDEVICE: return "device-side check failed";
        default: return "unknown status";
    }
}

extern "C" g4d_status g4d_set_stage_events(void *const *events, int32_t count) {
    if (!events) {
        g4d::g_stage_on = false;
        return G4D_OK;
    }
    if (count != g4d::kStageEvents) return G4D_EINVAL;
    for (int i = 0; i < g4d::kStageEvents; ++i) g4d::g_stage_events[i] = reinterpret_cast<hipEvent_t>(events[i]);
    g4d::g_stage_on = true;
    return G4D_OK;
}

extern "C" int32_t g4d_last_hip_error(void) { return g4d::g_last_hip_error; }

extern "C" const char *g4d_version(void) { return "g4d 0.1 gfx950"; }
