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

// ------------------------------------------------------------------ relayout
// Linear x-fastest stored brick -> 8^3 blocks (blocks x-fastest; the voxel order
// inside a block is the one of blk_x/blk_y/blk_z).  Four consecutive x-voxels from
// a multiple of 4 stay contiguous in both layouts, so the re-tiling is a copy of
// aligned 4-voxel runs, no transpose: a workgroup covers 64 x-voxels of 8 rows (y)
// in 2 z-slices, a wave a (y, y+1) x (z, z+1) pair of row pairs, so its reads are
// 4 contiguous row segments and, per block, its writes fill whole 64-byte
// sectors (4x2x2 voxels in FP32).  Padding voxels (beyond the stored dims) are
// zeroed at allocation and never read by the sampler.
template <typename E, typename V4>
__global__ __launch_bounds__(256) void relayout_kernel(const E* __restrict__ src, E* __restrict__ dst, int sx,
                                                       int sy, int sz, uint32_t bsy, uint32_t bsz, int nxt,
                                                       int nyt) {
  const int t = threadIdx.x;
  const int q = t & 15, r = t >> 4;  // 16 four-voxel runs x 16 (y, z) rows
  const int bxi = blockIdx.x % nxt;
  const int rest = blockIdx.x / nxt;
  const int yb = rest % nyt, zb = rest / nyt;
  const int x0 = bxi * 64 + 4 * q, y = yb * 8 + 2 * (r >> 2) + (r & 1), z = zb * 2 + ((r >> 1) & 1);
  if (x0 >= sx || y >= sy || z >= sz) return;
  const E* s = src + ((size_t)z * sy + y) * sx + x0;
  E* d = dst + ((size_t)blk_z(z, bsz) + blk_y(y, bsy) + blk_x(x0));
  if (x0 + 4 <= sx) {
    V4 v;
    v.x = s[0];
    v.y = s[1];
    v.z = s[2];
    v.w = s[3];
    *(V4*)d = v;  // x0 is a multiple of 4: the run is aligned and contiguous in the block
  } else {
    for (int i = 0; i < sx - x0; ++i) d[i] = s[i];
  }
}

// ------------------------------------------------------------------ macrocell ranges
// Macrocell m covers owned-relative voxels [mc m - 1, mc m + mc] per axis, clipped to
// the stored range (stored index = owned index + ghost_lo).  One workgroup of 8
// waves builds a run of up to (64 P - 2) / mc macrocells along x for one (my, mz):
// the waves split the (y, z) rows of the window, each reads its rows' x-span from
// the linear stored copy (coalesced, U rows in flight at once, addresses clamped
// into the window so every load is unconditional) and keeps a per-x-column
// min/max in registers (P columns per lane, P sized to the brick's width); the
// columns are combined in LDS and reduced over each macrocell's x-window.  Each
// element is read at most ((mc+2)/mc)^2 times in total (the y and z aprons).
constexpr int kMcWaves = 8;

template <typename T>
__device__ __forceinline__ float voxel_value(const T* p) {
  if constexpr (sizeof(T) == 2)
    return __half2float(*p);
  else
    return *p;
}

// Up to kMcJobs bricks of one element type and column count per launch; the
// workgroups of job j follow those of job j - 1.
struct McJob {
  const void* vox;
  float2* ranges;
  int sx, sy, sz, gx, gy, gz, mdx, mdy, mdz, per_chunk, chunks, blocks;
};
constexpr int kMcJobs = 16;
struct McJobs {
  McJob job[kMcJobs];
  int n;
};

template <typename T, int P, int U>
__global__ __launch_bounds__(64 * kMcWaves) void macrocell_kernel(McJobs jobs, int mc) {
  __shared__ float col_lo[64 * P], col_hi[64 * P];
  int bid = blockIdx.x, j = 0;
  while (j + 1 < jobs.n && bid >= jobs.job[j].blocks) bid -= jobs.job[j++].blocks;
  const McJob& J = jobs.job[j];
  const T* __restrict__ vox = (const T*)J.vox;
  const int sx = J.sx, sy = J.sy, sz = J.sz, gx = J.gx, gy = J.gy, gz = J.gz;
  const int mdx = J.mdx, mdy = J.mdy, chunks = J.chunks, per_chunk = J.per_chunk;
  const int c = bid % chunks;
  const int my = (bid / chunks) % mdy, mz = bid / (chunks * mdy);
  const int mx0 = c * per_chunk, mx1 = min(mdx, mx0 + per_chunk);
  const int xs = max(0, mc * mx0 - 1 + gx), xe = min(sx - 1, mc * mx1 + gx);
  const int wx = xe - xs + 1;
  const int y0 = max(0, mc * my - 1 + gy), y1 = min(sy - 1, mc * my + mc + gy);
  const int z0 = max(0, mc * mz - 1 + gz), z1 = min(sz - 1, mc * mz + mc + gz);
  const int wy = y1 - y0 + 1, rows = wy * (z1 - z0 + 1);
  for (int x = threadIdx.x; x < wx; x += 64 * kMcWaves) {
    col_lo[x] = INFINITY;
    col_hi[x] = -INFINITY;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float lo[P], hi[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    lo[j] = INFINITY;
    hi[j] = -INFINITY;
  }
  for (int r0 = wave; r0 < rows; r0 += kMcWaves * U) {
    float v[U][P];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = min(r0 + u * kMcWaves, rows - 1);
      const T* rowp = vox + ((size_t)(z0 + r / wy) * sy + (y0 + r % wy)) * sx + xs;
#pragma unroll
      for (int j = 0; j < P; ++j) v[u][j] = voxel_value(rowp + min(lane + 64 * j, wx - 1));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool row_ok = r0 + u * kMcWaves < rows;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const bool ok = row_ok && lane + 64 * j < wx;
        lo[j] = ok ? fminf(lo[j], v[u][j]) : lo[j];
        hi[j] = ok ? fmaxf(hi[j], v[u][j]) : hi[j];
      }
    }
  }
  // combine the waves' columns in LDS, one wave at a time
  for (int w = 0; w < kMcWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int x = lane + 64 * j;
        if (x < wx) {
          col_lo[x] = fminf(col_lo[x], lo[j]);
          col_hi[x] = fmaxf(col_hi[x], hi[j]);
        }
      }
    }
    __syncthreads();
  }
  // reduce each macrocell's x-window [mc mx - 1, mc mx + mc] (stored coordinates)
  for (int mx = mx0 + threadIdx.x; mx < mx1; mx += 64 * kMcWaves) {
    const int a0 = max(0, mc * mx - 1 + gx) - xs, a1 = min(sx - 1, mc * mx + mc + gx) - xs;
    float a = INFINITY, b = -INFINITY;
    for (int x = a0; x <= a1; ++x) {
      a = fminf(a, col_lo[x]);
      b = fmaxf(b, col_hi[x]);
    }
    J.ranges[((size_t)mz * mdy + my) * mdx + mx] = make_float2(a, b);
  }
}

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

// ------------------------------------------------------------------ host launchers
hipError_t launch_relayout(const void* src, void* dst, int elem_bytes, int sx, int sy, int sz, int bx, int by,
                           int bz, hipStream_t st) {
  (void)bz;
  const int nxt = (sx + 63) / 64, nyt = (sy + 7) / 8, nzt = (sz + 1) / 2;
  const uint32_t bsy = (uint32_t)kBlockVoxels * (uint32_t)bx, bsz = bsy * (uint32_t)by;
  const dim3 grid((unsigned)nxt * nyt * nzt);
  if (elem_bytes == 4)
    hipLaunchKernelGGL((relayout_kernel<uint32_t, uint4>), grid, dim3(256), 0, st, (const uint32_t*)src,
                       (uint32_t*)dst, sx, sy, sz, bsy, bsz, nxt, nyt);
  else
    hipLaunchKernelGGL((relayout_kernel<uint16_t, ushort4>), grid, dim3(256), 0, st, (const uint16_t*)src,
                       (uint16_t*)dst, sx, sy, sz, bsy, bsz, nxt, nyt);
  return hipGetLastError();
}

template <typename T, int P, int U>
static void launch_mc(const McBrick* bricks, const int* idx, int n, int mc, hipStream_t st) {
  for (int i0 = 0; i0 < n; i0 += kMcJobs) {
    McJobs jobs{};
    long long total = 0;
    for (int i = i0; i < std::min(n, i0 + kMcJobs); ++i) {
      const BrickG& b = bricks[idx[i]].view;
      McJob& J = jobs.job[jobs.n++];
      J.vox = bricks[idx[i]].linear;
      J.ranges = bricks[idx[i]].ranges;
      J.sx = b.sdim[0];
      J.sy = b.sdim[1];
      J.sz = b.sdim[2];
      J.gx = b.olo[0] - b.slo[0];
      J.gy = b.olo[1] - b.slo[1];
      J.gz = b.olo[2] - b.slo[2];
      J.mdx = b.mdim[0];
      J.mdy = b.mdim[1];
      J.mdz = b.mdim[2];
      J.per_chunk = (64 * P - 2) / mc;
      J.chunks = (b.mdim[0] + J.per_chunk - 1) / J.per_chunk;
      J.blocks = J.chunks * b.mdim[1] * b.mdim[2];
      total += J.blocks;
    }
    hipLaunchKernelGGL((macrocell_kernel<T, P, U>), dim3((unsigned)total), dim3(64 * kMcWaves), 0, st, jobs, mc);
  }
}

// Columns per lane: the narrowest instantiation that spans the brick's x-window.
static int mc_columns(const BrickG& b, int mc) {
  const int need = std::min(b.sdim[0], mc * b.mdim[0] + 2);
  for (int p : {2, 3, 5, 9})
    if (need <= 64 * p) return p;
  return 17;  // wider bricks: runs of x-chunks
}

template <typename T>
static void launch_mc_t(const McBrick* bricks, const std::vector<int>& ids, int mc, hipStream_t st) {
  for (int p : {2, 3, 5, 9, 17}) {
    std::vector<int> sel;
    for (int i : ids)
      if (mc_columns(bricks[i].view, mc) == p) sel.push_back(i);
    if (sel.empty()) continue;
    if (p == 2) launch_mc<T, 2, 4>(bricks, sel.data(), (int)sel.size(), mc, st);
    if (p == 3) launch_mc<T, 3, 4>(bricks, sel.data(), (int)sel.size(), mc, st);
    if (p == 5) launch_mc<T, 5, 4>(bricks, sel.data(), (int)sel.size(), mc, st);
    if (p == 9) launch_mc<T, 9, 2>(bricks, sel.data(), (int)sel.size(), mc, st);
    if (p == 17) launch_mc<T, 17, 1>(bricks, sel.data(), (int)sel.size(), mc, st);
  }
}

hipError_t launch_macrocells(const McBrick* bricks, int n, int mc, hipStream_t st) {
  std::vector<int> f32, f16;
  for (int i = 0; i < n; ++i) (bricks[i].f16 ? f16 : f32).push_back(i);
  if (!f32.empty()) launch_mc_t<float>(bricks, f32, mc, st);
  if (!f16.empty()) launch_mc_t<__half>(bricks, f16, mc, st);
  return hipGetLastError();
}

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

}  // namespace dpr
