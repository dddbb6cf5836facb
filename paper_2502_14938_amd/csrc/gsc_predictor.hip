// Reuse predictor: training and inference kernels.
#include "gsc_common.h"
#include "gsc_ctx.h"

namespace gsc {
void pred_free(gsc_ctx*) {}
}  // namespace gsc

extern "C" {
int gsc_predictor_load(gsc_ctx*, const float*, int64_t) { return GSC_E_INVALID_ARG; }
int gsc_predictor_get(gsc_ctx*, float*, int64_t) { return GSC_E_INVALID_ARG; }
int gsc_predictor_train(gsc_ctx*, const float*, const uint8_t*, int64_t, int32_t, int32_t, float, float, uint64_t,
                        float*) { return GSC_E_INVALID_ARG; }
int gsc_predictor_grad(gsc_ctx*, const float*, const float*, int64_t, float, float*, float*) { return GSC_E_INVALID_ARG; }
int gsc_predictor_infer(gsc_ctx*, const float*, int64_t, float*) { return GSC_E_INVALID_ARG; }
int gsc_predictor_features(gsc_ctx*, float*, int32_t*, int64_t, int64_t*) { return GSC_E_INVALID_ARG; }
}
