// World commit in one pass over each brick's linear stored copy: the 8^3-blocked
// copy the sampler reads and the macrocell (min, max) ranges.
//
// Macrocell m covers owned-relative voxels [mc m - 1, mc m + mc] per axis, clipped
// to the stored range (stored index = owned index + ghost_lo).  One workgroup
// handles one (my, mz) and a run of macrocells along x (all of them for bricks up
// to about 300 voxels wide): it reads the windows' rows, keeps per-x-column
// min/max in registers, combines the waves' columns in LDS and reduces each
// macrocell's x-window.  Windows overlap by two voxels per axis, so a voxel is
// read by up to 8 workgroups (mostly from L2); each voxel is written to the
// blocked copy by exactly one of them.  Write ownership goes by aligned groups:
// a 4-voxel x-run belongs to the workgroup whose x core [mc m + g, mc (m+1) + g)
// (the first core extended down to 0, the last up to the stored edge) holds its
// first voxel, and a (y, y+1) or (z, z+1) row pair to the one whose core holds its
// even row.  A wave copies 16 runs of a (y, y+1) x (z, z+1) row group, so its
// stores fill whole 64-byte sectors of the blocked layout.
#include <algorithm>
#include <vector>

#include "commit_span.h"
#include "kernels.h"

namespace dpr {

// Workgroups of 8 waves, held to 64 VGPRs (8 waves per SIMD) so that 4 of them
// fit a CU: the 2048 windows of eight 256^3-owned bricks run in two full rounds.
constexpr int kCmWaves = 8;

struct CmJob {
  const void* src;  // linear stored copy, x fastest
  void* dst;        // 8^3-blocked copy
  float2* ranges;
  int sx, sy, sz, gx, gy, gz, mdx, mdy, mdz, per_chunk, chunks, blocks;
  uint32_t bsy, bsz;
};
constexpr int kCmJobs = 16;
struct CmJobs {
  CmJob job[kCmJobs];
  int n;
};

template <typename E>
__device__ __forceinline__ float elem_value(E e) {
  if constexpr (sizeof(E) == 2)
    return __half2float(__ushort_as_half(e));
  else
    return __uint_as_float(e);
}

template <typename E, typename V4, int U>
__global__ __launch_bounds__(64 * kCmWaves) __attribute__((amdgpu_waves_per_eu(8))) void commit_kernel(CmJobs jobs, int mc) {
  __shared__ float part_lo[kCmWaves][kCmCols], part_hi[kCmWaves][kCmCols];
  int bid = blockIdx.x, j = 0;
  while (j + 1 < jobs.n && bid >= jobs.job[j].blocks) bid -= jobs.job[j++].blocks;
  const CmJob& J = jobs.job[j];
  const E* __restrict__ src = (const E*)J.src;
  uint32_t* __restrict__ dst = (uint32_t*)J.dst;
  const int sx = J.sx, sy = J.sy;
  const int c = bid % J.chunks;
  const int my = (bid / J.chunks) % J.mdy, mz = bid / (J.chunks * J.mdy);
  const int mx0 = c * J.per_chunk, mx1 = min(J.mdx, mx0 + J.per_chunk);
  const AxisSpan X = axis_span(mx0, mx1, J.mdx, mc, J.gx, sx, 4);
  const AxisSpan Y = axis_span(my, my + 1, J.mdy, mc, J.gy, sy, 2);
  const AxisSpan Z = axis_span(mz, mz + 1, J.mdz, mc, J.gz, J.sz, 2);
  const int nyp = (Y.le - Y.ls + 2) >> 1, nzp = (Z.le - Z.ls + 2) >> 1, groups = nyp * nzp;
  const int nxc = (X.le - X.ls + 64) >> 6;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane & 15, py = (lane >> 4) & 1, pz = lane >> 5;
  for (int xc = 0; xc < nxc; ++xc) {
    const int x0 = X.ls + 64 * xc + 4 * q;
    const int nrun = min(4, sx - x0);  // voxels of this run inside the brick (<= 0: none)
    const bool x_own = x0 >= X.cs && x0 < X.ce;
    float lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[k] = INFINITY;
      hi[k] = -INFINITY;
    }
    // this wave's row groups g = wave, wave + kCmWaves, ...: g = zi * nyp + yi,
    // stepped without divisions
    int yi = wave, zi = 0;
    while (yi >= nyp) {
      yi -= nyp;
      ++zi;
    }
    const bool x_ok = nrun > 0 && x0 <= X.le;
    for (int g0 = wave; g0 < groups; g0 += kCmWaves * U) {
      E v[U][4];
      bool live[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int yp = Y.ls + 2 * yi, zp = Z.ls + 2 * zi;
        const int y = yp + py, z = zp + pz;
        live[u] = g0 + u * kCmWaves < groups && x_ok && y <= Y.le && z <= Z.le;
#pragma unroll
        for (int k = 0; k < 4; ++k) v[u][k] = (E)0;
        if (live[u]) {
          const E* s = src + ((size_t)z * sy + y) * sx + x0;
          // (a row of the linear copy need not start on a 4-voxel boundary, so the
          // run is read voxel by voxel; neighbouring lanes read neighbouring runs)
          if (nrun == 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[u][k] = s[k];
          } else {
            for (int k = 0; k < nrun; ++k) v[u][k] = s[k];
          }
          if (x_own && yp >= Y.cs && yp < Y.ce && zp >= Z.cs && zp < Z.ce) {
            uint32_t* d = dst + ((size_t)blk_z(z, J.bsz) + blk_y(y, J.bsy) + blk_x(x0));
            uint32_t w[4];
            if constexpr (sizeof(E) == 2) {
              // FP16: element x holds the halves of voxels x and x + 1 (the brick's
              // last voxel has no x + 1; that half is never read)
              const E after = x0 + 4 < sx ? s[4] : v[u][3];
#pragma unroll
              for (int k = 0; k < 4; ++k) w[k] = (uint32_t)v[u][k] | ((uint32_t)(k < 3 ? v[u][k + 1] : after) << 16);
            } else {
#pragma unroll
              for (int k = 0; k < 4; ++k) w[k] = v[u][k];
            }
            if (nrun == 4) {  // x0 is a multiple of 4: an aligned run of the block
              *(uint4*)d = make_uint4(w[0], w[1], w[2], w[3]);
            } else {
              for (int k = 0; k < nrun; ++k) d[k] = w[k];
            }
          }
          live[u] = y >= Y.ws && y <= Y.we && z >= Z.ws && z <= Z.we;
        }
        yi += kCmWaves;
        while (yi >= nyp) {
          yi -= nyp;
          ++zi;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const bool ok = live[u] && k < nrun;
          const float f = elem_value(v[u][k]);
          lo[k] = ok ? fminf(lo[k], f) : lo[k];
          hi[k] = ok ? fmaxf(hi[k], f) : hi[k];
        }
      }
    }
    // the four (y, z) parities of a run sit 16 and 32 lanes apart
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], 16));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], 16));
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], 32));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], 32));
    }
    if (lane < 16) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        part_lo[wave][64 * xc + 4 * q + k] = lo[k];
        part_hi[wave][64 * xc + 4 * q + k] = hi[k];
      }
    }
  }
  __syncthreads();
  // reduce each macrocell's x-window over the waves' columns
  for (int mx = mx0 + (int)threadIdx.x; mx < mx1; mx += 64 * kCmWaves) {
    const int a0 = max(0, mc * mx - 1 + J.gx) - X.ls, a1 = min(sx - 1, mc * mx + mc + J.gx) - X.ls;
    float a = INFINITY, b = -INFINITY;
    for (int x = a0; x <= a1; ++x) {
#pragma unroll
      for (int w = 0; w < kCmWaves; ++w) {
        a = fminf(a, part_lo[w][x]);
        b = fmaxf(b, part_hi[w][x]);
      }
    }
    J.ranges[((size_t)mz * J.mdy + my) * J.mdx + mx] = make_float2(a, b);
  }
}

template <typename E, typename V4>
static void launch_commit_t(const McBrick* bricks, const std::vector<int>& ids, int mc, hipStream_t st) {
  for (size_t i0 = 0; i0 < ids.size(); i0 += kCmJobs) {
    CmJobs jobs{};
    long long total = 0;
    for (size_t i = i0; i < std::min(ids.size(), i0 + kCmJobs); ++i) {
      const McBrick& m = bricks[ids[i]];
      const BrickG& b = m.view;
      CmJob& J = jobs.job[jobs.n++];
      J.src = m.linear;
      J.dst = const_cast<void*>(b.data);
      J.ranges = m.ranges;
      J.sx = b.sdim[0];
      J.sy = b.sdim[1];
      J.sz = b.sdim[2];
      J.gx = b.olo[0] - b.slo[0];
      J.gy = b.olo[1] - b.slo[1];
      J.gz = b.olo[2] - b.slo[2];
      J.mdx = b.mdim[0];
      J.mdy = b.mdim[1];
      J.mdz = b.mdim[2];
      J.bsy = b.bsy;
      J.bsz = b.bsz;
      J.per_chunk = commit_per_chunk(b.sdim[0], b.olo[0] - b.slo[0], b.mdim[0], mc);
      J.chunks = (b.mdim[0] + J.per_chunk - 1) / J.per_chunk;
      J.blocks = J.chunks * b.mdim[1] * b.mdim[2];
      total += J.blocks;
    }
    hipLaunchKernelGGL((commit_kernel<E, V4, 2>), dim3((unsigned)total), dim3(64 * kCmWaves), 0, st, jobs, mc);
  }
}

hipError_t launch_commit(const McBrick* bricks, int n, int mc, hipStream_t st) {
  std::vector<int> f32, f16;
  for (int i = 0; i < n; ++i) (bricks[i].f16 ? f16 : f32).push_back(i);
  if (!f32.empty()) launch_commit_t<uint32_t, uint4>(bricks, f32, mc, st);
  if (!f16.empty()) launch_commit_t<uint16_t, ushort4>(bricks, f16, mc, st);
  return hipGetLastError();
}

}  // namespace dpr
