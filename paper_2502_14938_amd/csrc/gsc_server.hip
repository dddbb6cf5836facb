// Multi-viewer serving loop.
#include "gsc_common.h"
#include "gsc_ctx.h"

extern "C" {
int gsc_server_create(gsc_ctx*, int64_t, void*, gsc_server** out) { if (out) *out = nullptr; return GSC_E_INVALID_ARG; }
void gsc_server_destroy(gsc_server*) {}
int gsc_server_admit(gsc_server*, int32_t, int32_t) { return GSC_E_INVALID_ARG; }
int64_t gsc_server_viewer_bytes(gsc_server*, int32_t, int32_t) { return 0; }
int64_t gsc_server_submit(gsc_server*, int32_t, const gsc_camera*, const gsc_camera*, double, float*, float*) { return GSC_E_INVALID_ARG; }
int gsc_server_step(gsc_server*) { return GSC_E_INVALID_ARG; }
int gsc_server_poll(gsc_server*, int64_t*, double*, int32_t) { return 0; }
int gsc_server_leave(gsc_server*, int32_t) { return GSC_E_INVALID_ARG; }
}
