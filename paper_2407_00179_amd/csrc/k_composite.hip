// Sort-last compositor over K whole frames (dpr_composite).
//
// Fast path (one wave per 64 consecutive pixels, 4 waves per workgroup):
//   pass 1  read every source's depth for the 64 pixels (coalesced) and take the
//           nearest depth of each source over the tile with a wave reduction;
//   order   rank the sources by (nearest depth, id rank) -- the tile order;
//   pass 2  walk the sources in tile order, re-reading each lane's depth (now an
//           L2 / Infinity Cache hit) and fetching RGBA only for live fragments, and
//           composite front to back on the fly while checking, per pixel, that its
//           live fragments really arrive in (depth, id) order.
// Neighbouring pixels almost always share one order (convex bricks: a separating
// plane orders two bricks identically for every ray; per-rank depth slabs), so
// nothing is stored per pixel and no LDS staging limits occupancy.  A pixel whose
// fragments break the tile order is appended to a fix-up list and recomposited by
// the fully general per-wave sort (composite_wave), which gives the same bits.
#include "composite.h"
#include "device_common.h"
#include "kernels.h"

namespace dpr {

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}

template <int KMAX>
__global__ __launch_bounds__(256) void composite_fast_kernel(const CompTable* __restrict__ tab, int K, int P,
                                                             float4* __restrict__ out_rgba,
                                                             float* __restrict__ out_depth, int* __restrict__ fix_count,
                                                             int* __restrict__ fix_list) {
  __shared__ const float4* prgba[KMAX];
  __shared__ const float* pdepth[KMAX];
  __shared__ int prank[KMAX];
  __shared__ float rep[4][KMAX];
  __shared__ unsigned char order[4][KMAX];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = threadIdx.x; k < K; k += 256) {
    prgba[k] = tab->rgba[k];
    pdepth[k] = tab->depth[k];
    prank[k] = tab->idrank[k];
  }
  for (int k = lane; k < K; k += 64) order[wave][k] = (unsigned char)k;
  __syncthreads();
  const int p = (blockIdx.x * 4 + wave) * 64 + lane;
  const bool live_px = p < P;
  constexpr int B = KMAX < 16 ? KMAX : 16;
  // pass 1: nearest depth of each source over the tile
  for (int k0 = 0; k0 < K; k0 += B) {
    float z[B];
#pragma unroll
    for (int u = 0; u < B; ++u) z[u] = (live_px && k0 + u < K) ? pdepth[k0 + u][p] : INFINITY;
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const float m = wave_min(z[u]);
      if (lane == 0 && k0 + u < K) rep[wave][k0 + u] = m;
    }
  }
  __syncthreads();
  // tile order by (nearest depth, id rank)
  for (int k = lane; k < K; k += 64) {
    const float rk = rep[wave][k];
    const int ik = prank[k];
    int r = 0;
    for (int j = 0; j < K; ++j) {
      const float rj = rep[wave][j];
      r += (rj < rk) || (rj == rk && prank[j] < ik);
    }
    order[wave][r] = (unsigned char)k;
  }
  __syncthreads();
  // pass 2: composite in tile order, checking the per-pixel order
  float tr = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, ca = 0.f, zfirst = INFINITY;
  float lz = -INFINITY;
  int lr = -1;
  bool bad = !live_px;
  for (int i0 = 0; i0 < K; i0 += B) {
    int ku[B];
    float zu[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      ku[u] = (i0 + u < K) ? order[wave][i0 + u] : 0;
      zu[u] = (!bad && i0 + u < K) ? pdepth[ku[u]][p] : INFINITY;
    }
    float4 f[B];
#pragma unroll
    for (int u = 0; u < B; ++u) f[u] = (zu[u] < INFINITY) ? prgba[ku[u]][p] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (zu[u] < INFINITY && !bad) {
        const int r = prank[ku[u]];
        if (zu[u] > lz || (zu[u] == lz && r > lr)) {
          if (lr < 0) zfirst = zu[u];
          cr = fmaf(tr, f[u].x, cr);
          cg = fmaf(tr, f[u].y, cg);
          cb = fmaf(tr, f[u].z, cb);
          ca = fmaf(tr, f[u].w, ca);
          tr *= 1.f - f[u].w;
          lz = zu[u];
          lr = r;
        } else {
          bad = true;  // out of tile order: the general sort takes this pixel
        }
      }
    }
  }
  if (live_px) {
    if (bad) {
      const int slot = atomicAdd(fix_count, 1);
      fix_list[slot] = p;
    } else {
      out_rgba[p] = make_float4(cr, cg, cb, ca);
      out_depth[p] = zfirst;
    }
  }
}

// General path for the pixels of the fix-up list: one wave per 64 listed pixels,
// persistent over the list (its length is read on the device).
template <int KMAX>
__global__ __launch_bounds__(64) void composite_fixup_kernel(const CompTable* __restrict__ tab, int K,
                                                             float4* __restrict__ out_rgba,
                                                             float* __restrict__ out_depth,
                                                             const int* __restrict__ fix_count,
                                                             const int* __restrict__ fix_list) {
  __shared__ CompLDS<KMAX> s;
  __shared__ const float4* prgba[KMAX];
  __shared__ const float* pdepth[KMAX];
  const int lane = threadIdx.x;
  for (int k = lane; k < K; k += 64) {
    prgba[k] = tab->rgba[k];
    pdepth[k] = tab->depth[k];
  }
  __syncthreads();
  const int n = *fix_count;
  for (int base = blockIdx.x * 64; base < n; base += gridDim.x * 64) {
    const bool live = base + lane < n;
    const int p = live ? fix_list[base + lane] : 0;
    float4 c;
    float z;
    composite_wave<KMAX>(
        s, K, live, [&](int k) { return pdepth[k][p]; }, [&](int k) { return prgba[k][p]; },
        [&](int k) { return tab->idrank[k]; }, c, z);
    if (live) {
      out_rgba[p] = c;
      out_depth[p] = z;
    }
    __syncthreads();
  }
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

template <int KMAX>
static void launch_k(const CompTable* tab, int k, int n_pixels, float4* out_rgba, float* out_depth, int* fix_count,
                     int* fix_list, int fix_grid, hipStream_t st) {
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, fix_count);
  hipLaunchKernelGGL(composite_fast_kernel<KMAX>, dim3((n_pixels + 255) / 256), dim3(256), 0, st, tab, k, n_pixels,
                     out_rgba, out_depth, fix_count, fix_list);
  hipLaunchKernelGGL(composite_fixup_kernel<KMAX>, dim3(fix_grid), dim3(64), 0, st, tab, k, out_rgba, out_depth,
                     fix_count, fix_list);
}

hipError_t launch_composite(const CompTable* table_dev, int k, int n_pixels, float4* out_rgba, float* out_depth,
                            int* fix_count, int* fix_list, int fix_grid, hipStream_t st) {
  if (k <= 16)
    launch_k<16>(table_dev, k, n_pixels, out_rgba, out_depth, fix_count, fix_list, fix_grid, st);
  else if (k <= 64)
    launch_k<64>(table_dev, k, n_pixels, out_rgba, out_depth, fix_count, fix_list, fix_grid, st);
  else if (k <= 128)
    launch_k<128>(table_dev, k, n_pixels, out_rgba, out_depth, fix_count, fix_list, fix_grid, st);
  else
    launch_k<256>(table_dev, k, n_pixels, out_rgba, out_depth, fix_count, fix_list, fix_grid, st);
  return hipGetLastError();
}

}  // namespace dpr
