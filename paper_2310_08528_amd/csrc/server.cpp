// Serving loop (continuous batching) - not built yet in this revision.
#include "g4d_internal.h"

extern "C" {
g4d_status g4d_server_create(const g4d_server_config *, g4d_server **) { return G4D_EUNSUPPORTED; }
g4d_status g4d_server_add_scene(g4d_server *, const g4d_gaussians *, const g4d_planes *, const g4d_mlp *,
                                int32_t *) { return G4D_EUNSUPPORTED; }
g4d_status g4d_server_submit(g4d_server *, int32_t, const g4d_camera *, float, float *, uint64_t *) {
    return G4D_EUNSUPPORTED;
}
g4d_status g4d_server_wait(g4d_server *, uint64_t, double *) { return G4D_EUNSUPPORTED; }
g4d_status g4d_server_drain(g4d_server *) { return G4D_EUNSUPPORTED; }
g4d_status g4d_server_stats_get(g4d_server *, g4d_server_stats *) { return G4D_EUNSUPPORTED; }
g4d_status g4d_server_reset_stats(g4d_server *) { return G4D_EUNSUPPORTED; }
g4d_status g4d_server_destroy(g4d_server *) { return G4D_EUNSUPPORTED; }
}
