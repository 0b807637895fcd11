// Persistent batched renderer (work queue of (camera, brick, tile) items).
#include "runtime.hpp"

namespace dpr {

struct BatchState {};
void batch_state_free(BatchState* s) { delete s; }

}  // namespace dpr

using namespace dpr;

extern "C" {

dpr_status dpr_render_batch(dpr_world, const dpr_camera*, int32_t, dpr_frame*, uint32_t) {
  return fail(DPR_ERR_UNSUPPORTED, "dpr_render_batch: not built yet");
}
dpr_status dpr_autotune_batch(dpr_world, const dpr_camera*, int32_t, dpr_frame*, int32_t*, int32_t*) {
  return fail(DPR_ERR_UNSUPPORTED, "dpr_autotune_batch: not built yet");
}
dpr_status dpr_set_batch_tile(dpr_world, int32_t, int32_t) {
  return fail(DPR_ERR_UNSUPPORTED, "dpr_set_batch_tile: not built yet");
}

}  // extern "C"
