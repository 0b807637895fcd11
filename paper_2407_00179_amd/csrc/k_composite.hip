// Sort-last compositor: per pixel, sort the RGBA-z fragments with finite depth by
// (depth, id rank) and composite them front to back with the premultiplied "over"
// on all four channels: C += T rgba_i, T *= 1 - alpha_i.
//
// One wave owns 64 consecutive pixels.  All k depths of those pixels are staged in
// LDS with coalesced loads (4 B per fragment, the only bytes read for empty
// fragments).  The wave first orders the k frames by their nearest depth in the
// tile; neighbouring pixels almost always share that order (convex bricks, depth
// slabs), so each lane's insertion sort over its live fragments is nearly an
// append-only pass.  RGBA is then fetched only for live fragments, in sorted
// order, which keeps lanes on the same frame and the 16 B loads coalesced.
#include "device_common.h"
#include "kernels.h"

namespace dpr {

template <int KMAX>
__global__ __launch_bounds__(64) void composite_kernel(const CompTable* __restrict__ tab, int K, int P,
                                                       float4* __restrict__ out_rgba, float* __restrict__ out_depth) {
  __shared__ float zs[KMAX][65];
  __shared__ unsigned char lst[KMAX][64];
  __shared__ const float4* prgba[KMAX];
  __shared__ int prank[KMAX];
  __shared__ float rep[KMAX];
  __shared__ unsigned char order[KMAX];
  const int lane = threadIdx.x;
  const int p = blockIdx.x * 64 + lane;
  const bool live_px = p < P;
  for (int k = lane; k < K; k += 64) {
    prgba[k] = tab->rgba[k];
    prank[k] = tab->idrank[k];
    order[k] = (unsigned char)k;  // every slot holds a valid frame even if ranks collided
  }
  // 1. depths of the tile, coalesced per frame
  for (int k = 0; k < K; ++k) {
    const float* dp = tab->depth[k];
    zs[k][lane] = live_px ? dp[p] : INFINITY;
  }
  __syncthreads();
  // 2. tile order of the frames by (nearest depth in the tile, id rank)
  for (int k = lane; k < K; k += 64) {
    float m = INFINITY;
    for (int i = 0; i < 64; ++i) m = fminf(m, zs[k][i]);
    rep[k] = m;
  }
  __syncthreads();
  for (int k = lane; k < K; k += 64) {
    const float rk = rep[k];
    const int ik = prank[k];
    int rank = 0;
    for (int j = 0; j < K; ++j) {
      const float rj = rep[j];
      rank += (rj < rk) || (rj == rk && prank[j] < ik);
    }
    order[rank] = (unsigned char)k;
  }
  __syncthreads();
  // 3. per-lane sorted list of live fragments (insertion sort, nearly append-only)
  int n = 0;
  float lz = -INFINITY;
  int lr = -1;
  for (int i = 0; i < K; ++i) {
    const int k = order[i];
    const float z = zs[k][lane];
    if (!(z < INFINITY)) continue;
    const int r = prank[k];
    if (z > lz || (z == lz && r > lr)) {
      lst[n][lane] = (unsigned char)k;
      lz = z;
      lr = r;
    } else {
      int pos = n;
      while (pos > 0) {
        const int kk = lst[pos - 1][lane];
        const float zz = zs[kk][lane];
        if (zz < z || (zz == z && prank[kk] < r)) break;
        lst[pos][lane] = (unsigned char)kk;
        --pos;
      }
      lst[pos][lane] = (unsigned char)k;
    }
    ++n;
  }
  // 4. front-to-back over, RGBA fetched for live fragments only
  float tr = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, ca = 0.f;
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    float4 f[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) f[u] = prgba[lst[i + u][lane]][p];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      cr = fmaf(tr, f[u].x, cr);
      cg = fmaf(tr, f[u].y, cg);
      cb = fmaf(tr, f[u].z, cb);
      ca = fmaf(tr, f[u].w, ca);
      tr *= 1.f - f[u].w;
    }
  }
  for (; i < n; ++i) {
    const float4 f = prgba[lst[i][lane]][p];
    cr = fmaf(tr, f.x, cr);
    cg = fmaf(tr, f.y, cg);
    cb = fmaf(tr, f.z, cb);
    ca = fmaf(tr, f.w, ca);
    tr *= 1.f - f.w;
  }
  if (live_px) {
    out_rgba[p] = make_float4(cr, cg, cb, ca);
    out_depth[p] = n ? zs[lst[0][lane]][lane] : INFINITY;
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
