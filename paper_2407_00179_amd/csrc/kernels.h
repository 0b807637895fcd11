// Host-side launchers of the HIP kernels (all enqueue on the given stream).
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace dpr {

// Bytes past the end of a brick's linear copy that the commit may read (its run
// loads cover whole 8-voxel runs from an aligned dword); allocated, never used.
constexpr size_t kLinearSlack = 32;
// One brick of a commit: its linear stored copy, device view (view.data: the
// blocked copy to fill) and macrocell ranges to fill.
struct McBrick {
  const void* linear;
  BrickG view;
  float2* ranges;
  float2* partial;  // 2 per macrocell: scratch of the commit
  bool f16;
  bool half16;  // FP16 blocked copy of 2-byte voxels (else 4-byte voxel pairs)
};
// Blocked copy and macrocell ranges of several bricks in one pass over their
// linear stored copies.
hipError_t launch_commit(const McBrick* bricks, int n, int mc, int cu_count, hipStream_t st);
// Majorants of up to kMajJobs bricks in one launch (passed by value).
constexpr int kMajJobs = 32;
struct MajJobs {
  const float2* ranges[kMajJobs];
  float* maj[kMajJobs];
  int count[kMajJobs];
  int n;
  // with an iso-surface, a macrocell of majorant 0 gets its skip class: 0 (every
  // sample below iso), -1 (every sample at or above), 1 (must be sampled)
  int iso_on;
  float iso;
};
hipError_t launch_majorants(const MajJobs& jobs, const float4* tf, int ntf, float lo, float hi, hipStream_t st);
hipError_t launch_march(const SceneG& sc, const BrickG& b, const CamG& cam, const float4* tf, bool f16, bool skip,
                        float4* rgba, float* depth, int* count, hipStream_t st);
// Gather ceiling of the march (measurement): the march's loads for the first
// counts[p] logical samples of every pixel, with no dependence between samples.
hipError_t launch_gather_probe(const SceneG& sc, const BrickG& b, const CamG& cam, bool f16, const int* counts,
                               float* sink, hipStream_t st);

// Composite table: per fragment list entry, the frame pointers and the rank of
// its intrinsic id among the k ids (ties in depth are broken by that rank).
constexpr int kMaxFrags = 256;
struct CompTable {
  const float4* rgba[kMaxFrags];
  const float* depth[kMaxFrags];
  int idrank[kMaxFrags];
  // deep frames: per-pixel fragment counts of part k (null for flat frames) and
  // its layer capacity (counts are clamped to it)
  const int* count[kMaxFrags];
  int cap[kMaxFrags];
};
// fix_count / fix_list: device scratch for pixels whose fragments break the tile
// order (fix_count: two ints, zero on entry and left zero on exit; fix_list holds
// n_pixels ints); prior: kCompPriorFloats floats of scratch for the sampled nearest
// depth per source; cu_count: compute units of the device (sizes the grids).
constexpr int kCompPriorFloats = kMaxFrags * 8;
// Merge of deep frames: entry r of the table is part r (layer-major rgba/depth
// bases, counts, idrank = its place in rank order); parts <= kMaxFrags.
hipError_t launch_composite_deep(const CompTable* table_dev, int parts, int n_pixels, float4* out_rgba,
                                 float* out_depth, hipStream_t st);
hipError_t launch_composite(const CompTable* table_dev, int k, int n_pixels, float4* out_rgba, float* out_depth,
                            int* fix_count, int* fix_list, float* prior, int cu_count, hipStream_t st);

}  // namespace dpr
