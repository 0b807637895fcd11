// Host-side runtime objects behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dpr.h"
#include "kernels.h"

namespace dpr {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
dpr_status fail(dpr_status st, const char* fmt, ...);
dpr_status hip_fail(hipError_t e, const char* what);
bool log_enabled();

#define DPR_HIP(call)                                          \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return ::dpr::hip_fail(e_, #call);   \
  } while (0)

// Device and pinned host allocation, counted (dpr_alloc_stats) and with optional
// fault injection: DPR_FAULT_INJECT=alloc:N makes the N-th allocation of the
// process (of either kind) fail with DPR_ERR_OUT_OF_MEMORY.
dpr_status dev_alloc(void** p, size_t bytes, const char* what);
void dev_free(void* p);
dpr_status host_alloc(void** p, size_t bytes, const char* what);
void host_free(void* p);

struct CompEntry {
  CompTable* dev = nullptr;
  CompTable* host = nullptr;   // pinned; the async upload reads it
  uint64_t last_use = 0;
};

}  // namespace dpr

struct dpr_device_t {
  // references: the caller's handle plus one per live world, frame and deep frame;
  // the device is freed when the last one is released
  int refs = 1;
  int dev = 0;
  hipStream_t stream = nullptr;
  int cu_count = 0;
  int wave_size = 64;
  // composite tables keyed by (rgba ptr, depth ptr, id) of every part
  std::map<std::vector<uint64_t>, dpr::CompEntry> comp_cache;
  uint64_t use_clock = 0;
  // compositor fix-up scratch: list length + finish count (both zero between calls)
  // and a list of up to fix_cap pixel indices
  int* fix_count = nullptr;
  int* fix_list = nullptr;
  size_t fix_cap = 0;
  float* comp_prior = nullptr;  // sampled nearest depth per source (kCompPriorFloats)
  // FP64 sums of the transfer-function gradient across workgroups (dpr_render_backward)
  double* tf_grad64 = nullptr;
  // device address of the library's fixed scratch array on this GPU
  // (dpr_composite_noalloc), looked up when the handle is created
  void* noalloc_scratch = nullptr;
};

struct dpr_frame_t {
  dpr_device dev = nullptr;
  int w = 0, h = 0;
  float* rgba = nullptr;
  float* depth = nullptr;
  int* counts = nullptr;
  bool owned = false;
};

struct dpr_deep_frame_t {
  dpr_device dev = nullptr;
  int w = 0, h = 0, cap = 0;
  int rank = -1;  // set by dpr_render_deep
  int* counts = nullptr;
  float4* rgba = nullptr;
  float* depth = nullptr;
  int* ids = nullptr;
  bool owned = false;
};

namespace dpr {

struct Brick {
  int64_t olo[3], ohi[3];
  int32_t glo[3], ghi[3];
  int sdim[3];
  dpr_dtype dtype;
  void* linear = nullptr;     // stored region as given (x fastest)
  void* blocked = nullptr;    // 8^3-blocked copy used by the kernels
  int bdim[3] = {0, 0, 0};
  float2* ranges = nullptr;   // macrocell min/max
  float* maj = nullptr;       // macrocell majorant
  int mdim[3] = {0, 0, 0};
  int mc = 0;
  uint64_t maj_tf_version = 0;
  bool half16 = false;        // FP16 blocked copy of 2-byte voxels (else 4-byte voxel pairs)
  size_t elem() const { return dtype == DPR_F16 ? 2 : 4; }
  // bytes of one element of the blocked copy
  size_t blocked_elem() const { return dtype == DPR_F16 && half16 ? 2 : 4; }
  BrickG device_view(bool with_majorant, bool force_wide = false) const;
};

struct BatchState;  // persistent batched renderer (k_batch.hip)
void batch_state_free(BatchState*);
struct PathState;  // ray pools of the path tracer (k_path.hip)
void path_state_free(PathState*);

}  // namespace dpr

struct dpr_world_t {
  dpr_device dev = nullptr;
  int64_t dims[3] = {0, 0, 0};
  std::vector<dpr::Brick> bricks;
  bool committed = false;
  // transfer function
  float4* tf_dev = nullptr;
  int ntf = 0;
  float tf_lo = 0.f, tf_hi = 1.f, density = 0.f;
  bool tf_set = false;
  uint64_t tf_version = 0;  // bumped by every TF or iso-surface change (majorants are rebuilt)
  // opaque iso-surface
  bool iso_on = false;
  float iso = 0.f, iso_ka = 0.25f, iso_kd = 0.75f;
  // camera and parameters
  dpr_camera cam{};
  bool cam_set = false;
  dpr_render_params params{0.5f, 0.99f, 16, 0u};
  // partial frames of dpr_render_frame (one per brick)
  std::vector<dpr_frame> partials;
  dpr::BatchState* batch = nullptr;
  // per brick: the state of its partial renders through the persistent kernel
  std::vector<dpr::BatchState*> partial_batch;
  dpr::BatchState* last_batch = nullptr;  // the state of the last batched render
  dpr::PathState* path = nullptr;
  uint64_t geo_version = 1;  // bumped when a brick is added (invalidates batch item lists)
  uint64_t commit_version = 0;  // bumped by every commit (brick data may have changed)
  // pinned staging for transfer-function uploads; tf_ev marks the last upload
  float4* tf_host = nullptr;
  hipEvent_t tf_ev = nullptr;
  bool tf_ev_pending = false;
  int batch_tile_w = 8, batch_tile_h = 8;
};

namespace dpr {

CamG make_cam(const dpr_camera& c);
SceneG make_scene(const dpr_world_t* w);
dpr_status check_camera(const dpr_camera* c);
dpr_status ensure_majorants(dpr_world_t* w);
dpr_status render_frame_batched(dpr_world w, dpr_frame out);
dpr_status render_partial_batched(dpr_world w, int id, dpr_frame out);
dpr_status composite_frames(dpr_device dev, const dpr_frame* parts, const int32_t* ids, int32_t k, dpr_frame out);
// Largest frame (pixels) dpr_composite_noalloc takes: its fix-up list is sized
// for it (3840 x 2160 fits).
constexpr size_t kNoAllocMaxPixels = (size_t)1 << 23;
// Look up this GPU's copy of the fixed scratch array (the device is current).
dpr_status noalloc_setup(dpr_device d);
dpr_status comp_table(dpr_device dev, const std::vector<const float4*>& rgba, const std::vector<const float*>& depth,
                      const std::vector<int32_t>& ids, CompTable** out, const std::vector<const int*>* counts = nullptr,
                      const std::vector<int32_t>* caps = nullptr);

}  // namespace dpr
