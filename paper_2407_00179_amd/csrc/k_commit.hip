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
// even row.  A lane reads 8 consecutive voxels of a row with wide loads that need
// only 4-byte alignment, and a wave copies 16 such runs of a (y, y+1) x (z, z+1)
// row group, so its stores fill whole 64-byte sectors of the blocked layout.
#include <algorithm>
#include <vector>

#include "commit_span.h"
#include "kernels.h"

namespace dpr {

// Workgroups of 8 waves at up to 128 VGPRs (4 waves per SIMD, 2 workgroups per
// CU), each wave with the loads of 4 row groups in flight at once.
constexpr int kCmWaves = 8;
constexpr int kCmRowGroups = 4;

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

// A lane's x-run: 8 consecutive stored voxels of one row (two 4-voxel runs of the
// blocked layout).  A wave covers 16 runs (128 voxels) of a (y, y+1) x (z, z+1)
// row group.
constexpr int kRun = 8;
constexpr int kChunkX = 16 * kRun;

// Global loads that need only 4-byte alignment (rows of the linear copy start
// anywhere when a stored extent is odd).
typedef uint32_t U4a __attribute__((ext_vector_type(4), aligned(4)));
using GU32 = const uint32_t __attribute__((address_space(1)))*;
using GU4 = const U4a __attribute__((address_space(1)))*;

// The 8 voxels of a run: fetched raw (FP16: one 16-byte and one 4-byte load
// from the dword holding the first voxel cover its 9 halves; FP32: two 16-byte
// loads), then assembled into blocked elements.  FP16 element k is the pair
// (voxel k, voxel k + 1) as halves, cut out of neighbouring dwords with
// byte-align shifts; the brick's last voxel has no x + 1, so its pair repeats it
// (that half is never read).
template <typename E>
struct RawRun;
template <>
struct RawRun<uint16_t> {
  uint32_t d[5];
};
template <>
struct RawRun<uint32_t> {
  uint32_t d[kRun];
};

template <typename E>
__device__ __forceinline__ void fetch_run(const E* __restrict__ src, size_t e, RawRun<E>& r) {
  if constexpr (sizeof(E) == 2) {
    const GU32 p = (GU32)((const uint32_t*)src + (e >> 1));
    const U4a a = *(GU4)p;
    r.d[0] = a.x, r.d[1] = a.y, r.d[2] = a.z, r.d[3] = a.w;
    r.d[4] = p[4];
  } else {
    const GU4 p = (GU4)((const uint32_t*)src + e);
    const U4a a = p[0], b = p[1];
    r.d[0] = a.x, r.d[1] = a.y, r.d[2] = a.z, r.d[3] = a.w;
    r.d[4] = b.x, r.d[5] = b.y, r.d[6] = b.z, r.d[7] = b.w;
  }
}

template <typename E>
__device__ __forceinline__ void assemble_run(const RawRun<E>& r, bool odd, int x0, int sx, uint32_t w[kRun]) {
  if constexpr (sizeof(E) == 2) {
    const uint32_t* d = r.d;
    if (odd) {
#pragma unroll
      for (int k = 0; k < kRun; k += 2) {
        w[k] = __builtin_amdgcn_alignbyte(d[k / 2 + 1], d[k / 2], 2);
        w[k + 1] = d[k / 2 + 1];
      }
    } else {
#pragma unroll
      for (int k = 0; k < kRun; k += 2) {
        w[k] = d[k / 2];
        w[k + 1] = __builtin_amdgcn_alignbyte(d[k / 2 + 1], d[k / 2], 2);
      }
    }
#pragma unroll
    for (int k = 0; k < kRun; ++k)
      if (x0 + k + 1 >= sx) w[k] = (w[k] & 0xffffu) * 0x10001u;
  } else {
#pragma unroll
    for (int k = 0; k < kRun; ++k) w[k] = r.d[k];
  }
}

// Running per-column minimum and maximum of a lane's 8 columns.  FP16 keeps them
// as halves, two columns per register (the conversion to FP32 is exact, so the
// order of min/max and conversion does not matter): elements 0, 2, 4, 6 hold the
// voxel pairs (0, 1), (2, 3), (4, 5), (6, 7).  Columns at or beyond the brick's
// end may take any value; they are never read.
typedef _Float16 H2 __attribute__((ext_vector_type(2)));
template <typename E>
struct ColRange;
template <>
struct ColRange<uint16_t> {
  H2 lo[kRun / 2], hi[kRun / 2];
  __device__ void init() {
#pragma unroll
    for (int j = 0; j < kRun / 2; ++j) {
      lo[j] = H2{(_Float16)INFINITY, (_Float16)INFINITY};
      hi[j] = H2{(_Float16)-INFINITY, (_Float16)-INFINITY};
    }
  }
  __device__ void add(const uint32_t w[kRun]) {
#pragma unroll
    for (int j = 0; j < kRun / 2; ++j) {
      const H2 v = __builtin_bit_cast(H2, w[2 * j]);
      lo[j] = __builtin_elementwise_min(lo[j], v);
      hi[j] = __builtin_elementwise_max(hi[j], v);
    }
  }
  __device__ float get_lo(int k) const { return (float)lo[k / 2][k & 1]; }
  __device__ float get_hi(int k) const { return (float)hi[k / 2][k & 1]; }
};
template <>
struct ColRange<uint32_t> {
  float lo[kRun], hi[kRun];
  __device__ void init() {
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      lo[k] = INFINITY;
      hi[k] = -INFINITY;
    }
  }
  __device__ void add(const uint32_t w[kRun]) {
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      lo[k] = fminf(lo[k], __uint_as_float(w[k]));
      hi[k] = fmaxf(hi[k], __uint_as_float(w[k]));
    }
  }
  __device__ float get_lo(int k) const { return lo[k]; }
  __device__ float get_hi(int k) const { return hi[k]; }
};

// Store a 4-voxel run of the blocked copy (n of its voxels lie in the brick);
// dst + e is the run's first element.  4-byte elements (FP32 voxels, FP16 voxel
// pairs): the 4 elements w[0..3].  2-byte elements (FP16 voxels): the low halves
// of w[0..3], i.e. the halves of w[0] and w[2].
template <int EB>
__device__ __forceinline__ void store_run(void* __restrict__ dst, size_t e, const uint32_t* w, int n) {
  if constexpr (EB == 4) {
    uint32_t* d = (uint32_t*)dst + e;
    if (n >= 4) {  // an aligned run of the block
      *(uint4*)d = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
      for (int k = 0; k < n; ++k) d[k] = w[k];
    }
  } else {
    uint16_t* d = (uint16_t*)dst + e;
    if (n >= 4) {
      *(uint2*)d = make_uint2(w[0], w[2]);
    } else {
      for (int k = 0; k < n; ++k) d[k] = (uint16_t)(w[k] & 0xffffu);
    }
  }
}

template <typename E, int U, int EB>
__global__ __launch_bounds__(64 * kCmWaves) __attribute__((amdgpu_waves_per_eu(4))) void commit_kernel(CmJobs jobs, int mc) {
  __shared__ float part_lo[kCmWaves][kCmCols], part_hi[kCmWaves][kCmCols];
  int bid = blockIdx.x, j = 0;
  while (j + 1 < jobs.n && bid >= jobs.job[j].blocks) bid -= jobs.job[j++].blocks;
  const CmJob& J = jobs.job[j];
  const E* __restrict__ src = (const E*)J.src;
  void* __restrict__ dst = J.dst;
  const int sx = J.sx, sy = J.sy;
  const int c = bid % J.chunks;
  const int my = (bid / J.chunks) % J.mdy, mz = bid / (J.chunks * J.mdy);
  const int mx0 = c * J.per_chunk, mx1 = min(J.mdx, mx0 + J.per_chunk);
  const AxisSpan X = axis_span(mx0, mx1, J.mdx, mc, J.gx, sx, 4);
  const AxisSpan Y = axis_span(my, my + 1, J.mdy, mc, J.gy, sy, 2);
  const AxisSpan Z = axis_span(mz, mz + 1, J.mdz, mc, J.gz, J.sz, 2);
  const int nyp = (Y.le - Y.ls + 2) >> 1, nzp = (Z.le - Z.ls + 2) >> 1, groups = nyp * nzp;
  const int ncols = X.le - X.ls + 1;
  const int nxc = (ncols + kChunkX - 1) / kChunkX;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane & 15, py = (lane >> 4) & 1, pz = lane >> 5;
  for (int xc = 0; xc < nxc; ++xc) {
    const int x0 = X.ls + kChunkX * xc + kRun * q;
    const int nrun = min(kRun, sx - x0);  // voxels of this lane's run inside the brick (<= 0: none)
    // write ownership per 4-voxel run: the core holding the run's first voxel
    const bool own_a = x0 >= X.cs && x0 < X.ce, own_b = x0 + 4 >= X.cs && x0 + 4 < X.ce;
    ColRange<E> cr;
    cr.init();
    // this wave's row groups g = wave, wave + kCmWaves, ...: g = zi * nyp + yi,
    // stepped without divisions
    int yi = wave, zi = 0;
    while (yi >= nyp) {
      yi -= nyp;
      ++zi;
    }
    const bool x_ok = nrun > 0 && x0 <= X.le;
    for (int g0 = wave; g0 < groups; g0 += kCmWaves * U) {
      // the loads of U row groups are issued before any of them is used
      RawRun<E> raw[U];
      int yy[U], zz[U];
      bool live[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        yy[u] = Y.ls + 2 * yi;
        zz[u] = Z.ls + 2 * zi;
        const int y = yy[u] + py, z = zz[u] + pz;
        live[u] = g0 + u * kCmWaves < groups && x_ok && y <= Y.le && z <= Z.le;
        if (live[u]) fetch_run<E>(src, ((size_t)z * sy + y) * sx + x0, raw[u]);
        yi += kCmWaves;
        while (yi >= nyp) {
          yi -= nyp;
          ++zi;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!live[u]) continue;
        const int yp = yy[u], zp = zz[u], y = yp + py, z = zp + pz;
        uint32_t w[kRun];
        assemble_run<E>(raw[u], (((size_t)z * sy + y) * sx + x0) & 1, x0, sx, w);
        if ((own_a || own_b) && yp >= Y.cs && yp < Y.ce && zp >= Z.cs && zp < Z.ce) {
          const size_t e = (size_t)blk_z(z, J.bsz) + blk_y(y, J.bsy);
          if (own_a) store_run<EB>(dst, e + blk_x(x0), w, nrun);
          if (own_b) store_run<EB>(dst, e + blk_x(x0 + 4), w + 4, nrun - 4);
        }
        if (y >= Y.ws && y <= Y.we && z >= Z.ws && z <= Z.we) cr.add(w);
      }
    }
    // the four (y, z) parities of a run sit 16 and 32 lanes apart
    float lo[kRun], hi[kRun];
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      lo[k] = cr.get_lo(k);
      hi[k] = cr.get_hi(k);
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], 16));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], 16));
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], 32));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], 32));
    }
    if (lane < 16) {
#pragma unroll
      for (int k = 0; k < kRun; ++k) {
        const int col = kChunkX * xc + kRun * q + k;
        if (col < ncols) {
          part_lo[wave][col] = lo[k];
          part_hi[wave][col] = hi[k];
        }
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

template <typename E, int EB>
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
    hipLaunchKernelGGL((commit_kernel<E, kCmRowGroups, EB>), dim3((unsigned)total), dim3(64 * kCmWaves), 0, st, jobs, mc);
  }
}

hipError_t launch_commit(const McBrick* bricks, int n, int mc, hipStream_t st) {
  std::vector<int> f32, f16p, f16h;
  for (int i = 0; i < n; ++i) (bricks[i].f16 ? (bricks[i].half16 ? f16h : f16p) : f32).push_back(i);
  if (!f32.empty()) launch_commit_t<uint32_t, 4>(bricks, f32, mc, st);
  if (!f16p.empty()) launch_commit_t<uint16_t, 4>(bricks, f16p, mc, st);
  if (!f16h.empty()) launch_commit_t<uint16_t, 2>(bricks, f16h, mc, st);
  return hipGetLastError();
}

}  // namespace dpr
