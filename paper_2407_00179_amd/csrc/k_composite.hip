// Sort-last compositor over K whole frames (dpr_composite): one wave per 64
// consecutive pixels; the per-wave algorithm is composite_wave (composite.h).
#include "composite.h"
#include "device_common.h"
#include "kernels.h"

namespace dpr {

template <int KMAX>
__global__ __launch_bounds__(64) void composite_kernel(const CompTable* __restrict__ tab, int K, int P,
                                                       float4* __restrict__ out_rgba, float* __restrict__ out_depth) {
  __shared__ CompLDS<KMAX> s;
  __shared__ const float4* prgba[KMAX];
  __shared__ const float* pdepth[KMAX];
  const int lane = threadIdx.x;
  const int p = blockIdx.x * 64 + lane;
  const bool live_px = p < P;
  for (int k = lane; k < K; k += 64) {
    prgba[k] = tab->rgba[k];
    pdepth[k] = tab->depth[k];
  }
  __syncthreads();
  float4 c;
  float z;
  composite_wave<KMAX>(
      s, K, live_px, [&](int k) { return pdepth[k][p]; }, [&](int k) { return prgba[k][p]; },
      [&](int k) { return tab->idrank[k]; }, c, z);
  if (live_px) {
    out_rgba[p] = c;
    out_depth[p] = z;
  }
}

hipError_t launch_composite(const CompTable* table_dev, int k, int n_pixels, float4* out_rgba, float* out_depth,
                            hipStream_t st) {
  dim3 grid((n_pixels + 63) / 64), block(64);
  if (k <= 16)
    hipLaunchKernelGGL(composite_kernel<16>, grid, block, 0, st, table_dev, k, n_pixels, out_rgba, out_depth);
  else if (k <= 64)
    hipLaunchKernelGGL(composite_kernel<64>, grid, block, 0, st, table_dev, k, n_pixels, out_rgba, out_depth);
  else if (k <= 128)
    hipLaunchKernelGGL(composite_kernel<128>, grid, block, 0, st, table_dev, k, n_pixels, out_rgba, out_depth);
  else
    hipLaunchKernelGGL(composite_kernel<256>, grid, block, 0, st, table_dev, k, n_pixels, out_rgba, out_depth);
  return hipGetLastError();
}

}  // namespace dpr
