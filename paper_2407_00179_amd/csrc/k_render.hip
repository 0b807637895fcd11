// Brick ingest (8^3 relayout), macrocell ranges, transfer-function majorants and
// the per-brick emission-absorption ray march, for gfx950.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "device_common.h"
#include "kernels.h"
#include "majorant.h"
#include "march.h"

namespace dpr {

// ------------------------------------------------------------------ majorants
// Largest TF opacity over entries [floor(x_min) - 1, ceil(x_max) + 1] of the range's
// table coordinates x = clamp((v - lo)/(hi - lo), 0, 1) (N - 1), taken in FP32.
// One launch for the macrocells of up to kMajJobs bricks: thread m of the
// launch handles macrocell m of the concatenation of the jobs' grids.
__global__ __launch_bounds__(256) void majorant_kernel(MajJobs jobs, const float4* __restrict__ tf, int ntf,
                                                       float tf_lo, float tf_hi) {
  __shared__ float alpha[kMaxTF];
  for (int i = threadIdx.x; i < ntf; i += 256) alpha[i] = tf[i].w;
  __syncthreads();
  int m = blockIdx.x * 256 + threadIdx.x;
  int j = 0;
  while (j < jobs.n && m >= jobs.count[j]) m -= jobs.count[j++];
  if (j >= jobs.n) return;
  const float2 r = jobs.ranges[j][m];
  float a = tf_majorant(r, alpha, ntf, tf_lo, tf_hi);
  if (jobs.iso_on && a == 0.f) {
    // a margin of 1e-6 of the range's magnitude covers the rounding of FP32
    // trilinear values (a few ulps); no contraction, so the class is exact
    const float mg = __fmul_rn(1e-6f, fmaxf(fabsf(r.x), fabsf(r.y)));
    if (r.y < __fsub_rn(jobs.iso, mg))
      a = 0.f;
    else if (r.x > __fadd_rn(jobs.iso, mg))
      a = -1.f;
    else
      a = 1.f;
  }
  jobs.maj[j][m] = a;
}

// Plain per-brick launch: one thread per pixel, 16x16 tiles as four 8x8 waves,
// tiles assigned so that each XCD (round-robin workgroup dispatch) walks one
// contiguous band of the screen and keeps its part of the brick in its own L2.
template <typename T, bool SKIP, bool WIDE, bool ISO>
__global__ __launch_bounds__(256) void march_kernel(SceneG sc, BrickG b, CamG cam, const float4* __restrict__ tf,
                                                    float4* __restrict__ out_rgba, float* __restrict__ out_depth,
                                                    int* __restrict__ out_count, int tiles_x, int n_tiles) {
  extern __shared__ float4 tf_lds[];
  float4* tfb = tf_lds;
  float4* tfs = tf_lds + sc.ntf;
  stage_tf(tf, sc.ntf, tfb, tfs, threadIdx.x, 256);
  __syncthreads();
  const int nb = gridDim.x;
  const int per = (nb + 7) >> 3;
  const int bid = blockIdx.x;
  const int tile = (bid & 7) * per + (bid >> 3);
  if (tile >= n_tiles) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = (tile % tiles_x) * 16 + (wave & 1) * 8 + (lane & 7);
  const int py = (tile / tiles_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
  if (px >= cam.W || py >= cam.H) return;
  double d[3];
  camera_ray(cam, px, py, d);
  RayState r;
  const size_t p = (size_t)py * cam.W + px;
  if (ray_start<T, WIDE, ISO>(sc, b, cam.eye, d, r)) {
    ray_advance<T, SKIP, WIDE, ISO>(sc, b, tfb, tfs, r, 0x7fffffff);
    out_rgba[p] = make_float4(r.cr, r.cg, r.cb, 1.f - r.T);
    out_depth[p] = (float)r.t_in;
  } else {
    r.n = 0;
    out_rgba[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    out_depth[p] = INFINITY;
  }
  if (out_count) out_count[p] = r.n;
}

// Gather ceiling of the march (a measurement, not part of rendering): per pixel,
// the march's own lattice sample points over its first n logical samples (n
// from a march's per-pixel sample counts), the same skip rule and the same
// 8-voxel loads, but no transfer function, no compositing and no dependence
// between samples.  Each ray's samples are cut into kProbeSlots contiguous slices
// handled by different threads (grid y), and every thread keeps the loads of
// kProbeUnroll samples in flight, so no ray's length bounds the probe.  A skipped
// sample (macrocell majorant 0) re-reads the previous point, which the cache
// already holds.  The sum of the loaded values is added to sink[p].
constexpr int kProbeUnroll = 4;
constexpr int kProbeSlots = 16;
template <typename T, bool WIDE>
__global__ __launch_bounds__(256) void gather_probe_kernel(SceneG sc, BrickG b, CamG cam,
                                                           const int* __restrict__ counts, float* __restrict__ sink,
                                                           int tiles_x, int n_tiles) {
  // consecutive tiles go to consecutive workgroups, so the XCDs (dealt workgroups
  // in turn) share every part of the screen, however little of it the brick covers
  const int tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = (tile % tiles_x) * 16 + (wave & 1) * 8 + (lane & 7);
  const int py = (tile / tiles_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
  if (px >= cam.W || py >= cam.H) return;
  const size_t p = (size_t)py * cam.W + px;
  const int n = counts[p];
  const int slot = blockIdx.y;
  const int k0 = (int)((int64_t)n * slot / kProbeSlots), k1 = (int)((int64_t)n * (slot + 1) / kProbeSlots);
  float acc = 0.f;
  double d[3];
  camera_ray(cam, px, py, d);
  RayState r;
  if (k1 > k0 && ray_begin(sc, b, cam.eye, d, r)) {
    const int64_t half = 0x80000000ll;
    int64_t last[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) last[a] = r.p[a] + (int64_t)k0 * r.dp[a];
    for (int i = k0; i < k1; i += kProbeUnroll) {
      int64_t q[kProbeUnroll][3];
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) {
        const int k = min(i + u, k1 - 1);
        int m[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          q[u][a] = r.p[a] + (int64_t)k * r.dp[a];
          const int cell = (int)((q[u][a] + half) >> 32);
          m[a] = min(max((cell - b.olo[a]) >> b.mc_shift, 0), b.mdim[a] - 1);
        }
        const bool empty = b.majorant && ld_global(b.majorant, (m[2] * b.mdim[1] + m[1]) * b.mdim[0] + m[0]) == 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          q[u][a] = empty ? last[a] : q[u][a];
          last[a] = q[u][a];
        }
      }
      float v[kProbeUnroll];
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) {
        Gather<T> g;
        gather<T, WIDE>(sc, b, q[u], g);
        v[u] = ((g.v[0] + g.v[1]) + (g.v[2] + g.v[3])) + ((g.v[4] + g.v[5]) + (g.v[6] + g.v[7]));
      }
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) acc += v[u];
    }
  }
  if (k1 > k0) atomicAdd(&sink[p], acc);
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_majorants(const MajJobs& jobs, const float4* tf, int ntf, float lo, float hi, hipStream_t st) {
  long long total = 0;
  for (int j = 0; j < jobs.n; ++j) total += jobs.count[j];
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(majorant_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, jobs, tf, ntf, lo, hi);
  return hipGetLastError();
}

hipError_t launch_march(const SceneG& sc, const BrickG& b, const CamG& cam, const float4* tf, bool f16, bool skip,
                        float4* rgba, float* depth, int* count, hipStream_t st) {
  int tx = (cam.W + 15) / 16, ty = (cam.H + 15) / 16;
  int n_tiles = tx * ty;
  int nb = ((n_tiles + 7) / 8) * 8;
  dim3 grid(nb), block(256);
  size_t lds = 2 * sizeof(float4) * (size_t)sc.ntf;
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, grid, block, lds, st, sc, b, cam, tf, rgba, depth, count, tx, n_tiles);
  };
  auto by_wide = [&](auto t, auto sk, auto iso) {
    using T = decltype(t);
    constexpr bool S = decltype(sk)::value, I = decltype(iso)::value;
    b.wide ? go(march_kernel<T, S, true, I>) : go(march_kernel<T, S, false, I>);
  };
  auto by_iso = [&](auto t, auto sk) {
    sc.iso_on ? by_wide(t, sk, std::true_type{}) : by_wide(t, sk, std::false_type{});
  };
  auto by_skip = [&](auto t) { skip ? by_iso(t, std::true_type{}) : by_iso(t, std::false_type{}); };
  if (f16)
    by_skip(__half{});
  else
    by_skip(float{});
  return hipGetLastError();
}

hipError_t launch_gather_probe(const SceneG& sc, const BrickG& b, const CamG& cam, bool f16, const int* counts,
                               float* sink, hipStream_t st) {
  int tx = (cam.W + 15) / 16, ty = (cam.H + 15) / 16;
  int n_tiles = tx * ty;
  int nb = ((n_tiles + 7) / 8) * 8;
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(nb, kProbeSlots), dim3(256), 0, st, sc, b, cam, counts, sink, tx, n_tiles);
  };
  if (f16)
    b.wide ? go(gather_probe_kernel<__half, true>) : go(gather_probe_kernel<__half, false>);
  else
    b.wide ? go(gather_probe_kernel<float, true>) : go(gather_probe_kernel<float, false>);
  return hipGetLastError();
}

}  // namespace dpr
