// Differentiable forward render and adjoint ray march.
#include "runtime.hpp"

using namespace dpr;

extern "C" {

dpr_status dpr_train_workspace_size(const int64_t*, const dpr_camera*, int32_t, float, size_t*) {
  return fail(DPR_ERR_UNSUPPORTED, "dpr_train_workspace_size: not built yet");
}
dpr_status dpr_render_train_forward(dpr_device, const float*, const int64_t*, const float*, int32_t, float, float,
                                    float, const dpr_render_params*, const dpr_camera*, int32_t, float*, float*,
                                    void*, size_t) {
  return fail(DPR_ERR_UNSUPPORTED, "dpr_render_train_forward: not built yet");
}
dpr_status dpr_render_backward(dpr_device, const float*, const int64_t*, const float*, int32_t, float, float, float,
                               const dpr_render_params*, const dpr_camera*, int32_t, const float*, const void*,
                               size_t, float*, float*) {
  return fail(DPR_ERR_UNSUPPORTED, "dpr_render_backward: not built yet");
}

}  // extern "C"
