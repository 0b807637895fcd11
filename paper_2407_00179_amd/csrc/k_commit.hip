// World commit in one pass over each brick's linear stored copy: the 8^3-blocked
// copy the sampler reads and the macrocell (min, max) ranges.
//
// Macrocell m covers owned-relative voxels [mc m - 1, mc m + mc] per axis, clipped
// to the stored range (stored index = owned index + ghost_lo).  One wave handles
// one aligned span of 128 stored columns (whole cache lines, read by no other
// wave), one y macrocell and a segment of z macrocells, and streams through z one
// macrocell core at a time: every row it reads is read once, copied to the
// blocked layout if this wave owns it, and folded into the running per-column
// (min, max) of each macrocell window it lies in -- at most three at a time (the
// previous, current and next macrocell), kept in registers.  When a stage ends,
// the previous macrocell's window is complete: its columns are combined across
// the lanes of the four (y, z) parities, and each x-window's part in the span is
// reduced through a small wave-private LDS row into one of the macrocell's two
// partial ranges (a window meets one or two spans); a small second kernel takes
// their union.  Only the one-row y aprons of neighbouring macrocells are read
// twice; a workgroup's four waves (consecutive y macrocells) meet at a barrier
// after every z stage and sweep their rows in opposite directions (odd y
// macrocells downwards), so the rows two neighbours share are read by both in
// the same batch and the second read mostly hits in L2.  Write ownership: every
// column belongs to its span, and a (y, y+1) or (z, z+1) row pair to the
// macrocell whose core [mc m + g, mc (m+1) + g) (the first core extended down to
// 0, the last up to the stored edge) holds its even row.  A lane reads 8
// consecutive voxels of a row with wide loads that need only 4-byte alignment;
// the rows are visited in quads of 4 x 4 (y, z) rows aligned to the blocked
// layout, so the stores of one batch fill whole 64-element groups of it.
#include <algorithm>
#include <cmath>
#include <vector>

#include "commit_span.h"
#include "kernels.h"

namespace dpr {

// A lane's x-run: 8 consecutive stored voxels of one row (two 4-voxel runs of the
// blocked layout).  A wave covers 16 runs (128 voxels) of a (y, y+1) x (z, z+1)
// row group.
constexpr int kRun = 8;
static_assert(16 * kRun == kCmCols, "a wave's 16 runs span the chunk");

// Global loads that need only 4-byte alignment (rows of the linear copy start
// anywhere when a stored extent is odd).
typedef uint32_t U4a __attribute__((ext_vector_type(4), aligned(4)));
using GU32 = const uint32_t __attribute__((address_space(1)))*;
using GU4 = const U4a __attribute__((address_space(1)))*;

// The 8 voxels of a run: fetched raw (FP16: one 16-byte load from the dword
// holding the first voxel, plus the next dword when the run starts on an odd
// voxel or the pairs below need voxel 8; FP32: two 16-byte loads), then
// assembled into 32-bit words.  FP16 word k is the pair (voxel k, voxel k + 1)
// as halves, cut out of neighbouring dwords with byte-align shifts; the even
// words carry the run's 8 voxels.  For the pair layout (EB = 4) the brick's last
// voxel has no x + 1, so its pair repeats it (that half is never read).
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

template <typename E, int EB>
__device__ __forceinline__ void fetch_run(const E* __restrict__ src, size_t e, RawRun<E>& r) {
  if constexpr (sizeof(E) == 2) {
    const GU32 p = (GU32)((const uint32_t*)src + (e >> 1));
    const U4a a = *(GU4)p;
    r.d[0] = a.x, r.d[1] = a.y, r.d[2] = a.z, r.d[3] = a.w;
    if constexpr (EB == 4)
      r.d[4] = p[4];
    else
      r.d[4] = (e & 1) ? p[4] : 0u;
  } else {
    const GU4 p = (GU4)((const uint32_t*)src + e);
    const U4a a = p[0], b = p[1];
    r.d[0] = a.x, r.d[1] = a.y, r.d[2] = a.z, r.d[3] = a.w;
    r.d[4] = b.x, r.d[5] = b.y, r.d[6] = b.z, r.d[7] = b.w;
  }
}

template <typename E, int EB>
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
    if constexpr (EB == 4) {
#pragma unroll
      for (int k = 0; k < kRun; ++k)
        if (x0 + k + 1 >= sx) w[k] = (w[k] & 0xffffu) * 0x10001u;
    }
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

// One wave per (x-span, y macrocell, z-segment); a workgroup holds the waves of
// kCmWaves consecutive y macrocells.  At up to 128 VGPRs a CU runs 16 such waves,
// each with the loads of one quad of row groups in flight at once (FP32: half a
// quad).
constexpr int kCmWaves = 4;
constexpr int kCmWavesPerCu = 16;
template <typename E, int EB>
constexpr int cm_batch() {
  return sizeof(E) == 4 ? 2 : 4;
}
// 2-byte layout: a quad's 16 rows of a lane's two 4-voxel runs are two whole
// 128-byte lines of the blocked copy (64 elements: 4 x, 4 y, 4 z).  A quad the
// wave owns entirely is staged in LDS and stored as whole lines, 8 lanes a line,
// so no line reaches the L2 in pieces.  LDS chunks of 16 bytes are swizzled
// within a line by the run's lane to spread the writes over the banks.
constexpr int kStageQuadU4 = 2 * 16 * 8;  // uint4 per staged quad: 32 lines of 8 chunks
__device__ __forceinline__ int stage_chunk(int line, int chunk) { return line * 8 + (chunk ^ ((line >> 1) & 7)); }

struct CmJob {
  const void* src;  // linear stored copy, x fastest
  void* dst;        // 8^3-blocked copy
  float2* partial;  // 2 per macrocell
  int sx, sy, sz, gx, gy, gz, mdx, mdy, mdz;
  int spans, ygroups, seg, segs, blocks;
  uint32_t bsy, bsz;
};
constexpr int kCmJobs = 16;
struct CmJobs {
  CmJob job[kCmJobs];
  int n, blocks, per_xcd;
};

// Window [lo, hi] of z macrocell m when it lies in the segment [m0, m1), else empty.
__device__ __forceinline__ void z_window(int m, int m0, int m1, int mc, int g, int n, int& lo, int& hi) {
  if (m < m0 || m >= m1) {
    lo = 1;
    hi = 0;
  } else {
    lo = max(0, mc * m - 1 + g);
    hi = min(n - 1, mc * m + mc + g);
  }
}

template <typename E, int U, int EB>
__global__ __launch_bounds__(64 * kCmWaves) __attribute__((amdgpu_waves_per_eu(4))) void commit_kernel(CmJobs jobs, int mc) {
  static_assert(4 % U == 0 || U % 4 == 0, "batches hold whole quads or whole fractions of one");
  static_assert(EB == 4 || U % 4 == 0, "the 2-byte layout stages whole quads");
  constexpr int kQuads = EB == 2 ? U / 4 : 0;  // staged quads of a batch
  __shared__ float part[kCmWaves][2][kCmCols];
  __shared__ uint4 stage[kCmWaves][kQuads > 0 ? kQuads * kStageQuadU4 : 1];
  // workgroups reach the 8 XCDs in turn: give each XCD a contiguous run of the work
  const int t = (int)(blockIdx.x & 7) * jobs.per_xcd + (int)(blockIdx.x >> 3);
  if (t >= jobs.blocks) return;
  int bid = t, j = 0;
  while (j + 1 < jobs.n && bid >= jobs.job[j].blocks) bid -= jobs.job[j++].blocks;
  const CmJob& J = jobs.job[j];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int my0 = (bid % J.ygroups) * kCmWaves + wave;
  const bool active = my0 < J.mdy;  // an idle wave still meets the workgroup's stage barriers
  const int my = active ? my0 : J.mdy - 1;
  const bool rev = my & 1;          // odd y macrocells sweep their quads downwards
  const int k = (bid / J.ygroups) % J.spans, sg = bid / (J.ygroups * J.spans);
  const E* __restrict__ src = (const E*)J.src;
  void* __restrict__ dst = J.dst;
  const int sx = J.sx, sy = J.sy, sz = J.sz;
  const int xs0 = kCmCols * k, xs1 = min(sx - 1, xs0 + kCmCols - 1);
  const XCells XC = xspan_cells(k, J.mdx, mc, J.gx, sx);
  const int mz0 = sg * J.seg, mz1 = min(J.mdz, mz0 + J.seg);
  const AxisSpan Y = axis_span(my, my + 1, J.mdy, mc, J.gy, sy, 2);
  // row pairs of the y range in quads aligned to 4 rows (a quad's 4 x 4 rows of
  // (y, z) and a lane's 4-voxel run fill whole 64-element groups of the blocked layout)
  const int yq0 = Y.ls & ~3, nyq = ((Y.le - yq0) >> 2) + 1;
  // rows of the segment's macrocell windows
  const int zw0 = max(0, mc * mz0 - 1 + J.gz), zw1 = min(sz - 1, mc * mz1 + J.gz);

  const int q = lane & 15, py = (lane >> 4) & 1, pz = lane >> 5;
  const int x0 = xs0 + kRun * q;
  const int nrun = min(kRun, sx - x0);  // voxels of this lane's run inside the brick (<= 0: none)
  const bool x_ok = nrun > 0;
  float* lds_lo = part[wave][0];
  float* lds_hi = part[wave][1];
  uint4* stg = stage[wave];
  const bool full_span = xs0 + kCmCols <= sx;  // every lane holds a whole run

  // column ranges of the windows of z macrocells s - 1 (A), s (B) and s + 1 (C)
  ColRange<E> A, B, C;
  A.init();
  B.init();
  C.init();
  for (int s = mz0 - 1; s <= mz1; ++s) {
    const ZStage st = z_stage(s, mz0, mz1, J.mdz, mc, J.gz, sz);
    int a0, a1, b0, b1, c0, c1;
    z_window(s - 1, mz0, mz1, mc, J.gz, sz, a0, a1);
    z_window(s, mz0, mz1, mc, J.gz, sz, b0, b1);
    z_window(s + 1, mz0, mz1, mc, J.gz, sz, c0, c1);
    const int zq0 = st.lo & ~3;
    const int items = active && st.hi > st.lo ? 4 * (((st.hi - 1 - zq0) >> 2) + 1) * nyq : 0;  // 4 row groups a quad
    int yqi = 0, zqi = 0;  // quad of the batch's first row group (quads y fastest)
    for (int i0 = 0; i0 < items; i0 += U) {
      // the loads of U row groups are issued before any of them is used
      RawRun<E> raw[U];
      int yy[U], zz[U];
      bool live[U];
      int yq = yqi, zq = zqi;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int sub = (i0 + u) & 3;
        if (u > 0 && sub == 0 && ++yq == nyq) {
          yq = 0;
          ++zq;
        }
        yy[u] = yq0 + 4 * (rev ? nyq - 1 - yq : yq) + 2 * (sub & 1);
        zz[u] = zq0 + 4 * zq + 2 * (sub >> 1);
        const int y = yy[u] + py, z = zz[u] + pz;
        const bool win = y >= Y.ws && y <= Y.we && z >= zw0 && z <= zw1;
        const bool own = st.own && yy[u] >= Y.cs && yy[u] < Y.ce;
        live[u] = i0 + u < items && x_ok && yy[u] >= Y.ls && y <= Y.le && zz[u] >= st.lo && zz[u] < st.hi && z < sz &&
                  (win || own);
        if (live[u]) fetch_run<E, EB>(src, ((size_t)z * sy + y) * sx + x0, raw[u]);
      }
      if (((i0 + U) & 3) == 0 && ++yq == nyq) {
        yq = 0;
        ++zq;
      }
      yqi = yq;
      zqi = zq;
      // quads of the batch that this wave writes entirely (wave-uniform)
      bool staged[kQuads > 0 ? kQuads : 1];
#pragma unroll
      for (int b = 0; b < kQuads; ++b) {
        const int y4 = yy[4 * b], z4 = zz[4 * b];
        staged[b] = full_span && st.own && i0 + 4 * b < items && y4 >= Y.cs && y4 + 2 < Y.ce && y4 + 3 < sy &&
                    z4 >= st.lo && z4 + 2 < st.hi && z4 + 3 < sz;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!live[u]) continue;
        const int y = yy[u] + py, z = zz[u] + pz;
        uint32_t w[kRun];
        assemble_run<E, EB>(raw[u], (((size_t)z * sy + y) * sx + x0) & 1, x0, sx, w);
        if (kQuads > 0 && staged[u / 4]) {
          // element group (y0, z0, y1, z1) of the two lines of this lane's runs
          const int gi = py + 2 * pz + 4 * (u & 3);
          uint2* q2 = (uint2*)(stg + (u / 4) * kStageQuadU4);
          q2[2 * stage_chunk(2 * q, gi >> 1) + (gi & 1)] = make_uint2(w[0], w[2]);
          q2[2 * stage_chunk(2 * q + 1, gi >> 1) + (gi & 1)] = make_uint2(w[4], w[6]);
        } else if (st.own && yy[u] >= Y.cs && yy[u] < Y.ce) {
          const size_t e = (size_t)blk_z(z, J.bsz) + blk_y(y, J.bsy);
          store_run<EB>(dst, e + blk_x(x0), w, nrun);
          if (nrun > 4) store_run<EB>(dst, e + blk_x(x0 + 4), w + 4, nrun - 4);
        }
        if (y >= Y.ws && y <= Y.we) {
          if (z >= a0 && z <= a1) A.add(w);
          if (z >= b0 && z <= b1) B.add(w);
          if (z >= c0 && z <= c1) C.add(w);
        }
      }
      // staged quads out as whole lines: line li = 2 q + run, 16-byte chunk c
#pragma unroll
      for (int b = 0; b < kQuads; ++b) {
        if (!staged[b]) continue;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const size_t e = (size_t)blk_z(zz[4 * b], J.bsz) + blk_y(yy[4 * b], J.bsy);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int li = 8 * i + (lane >> 3), c = lane & 7;
          const uint4 v = stg[b * kStageQuadU4 + stage_chunk(li, c)];
          *(uint4*)((uint16_t*)dst + e + blk_x(xs0 + 4 * li) + 8 * c) = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    if (active && s - 1 >= mz0) {
      // macrocell s - 1's window is complete: combine the four (y, z) parities of
      // each column (16 and 32 lanes apart), then reduce each x-window's part in
      // this span
      float lo[kRun], hi[kRun];
#pragma unroll
      for (int kk = 0; kk < kRun; ++kk) {
        lo[kk] = A.get_lo(kk);
        hi[kk] = A.get_hi(kk);
        lo[kk] = fminf(lo[kk], __shfl_xor(lo[kk], 16));
        hi[kk] = fmaxf(hi[kk], __shfl_xor(hi[kk], 16));
        lo[kk] = fminf(lo[kk], __shfl_xor(lo[kk], 32));
        hi[kk] = fmaxf(hi[kk], __shfl_xor(hi[kk], 32));
      }
      if (lane < 16) {
#pragma unroll
        for (int kk = 0; kk < kRun; ++kk) {
          if (kk < nrun) {
            lds_lo[kRun * q + kk] = lo[kk];
            lds_hi[kRun * q + kk] = hi[kk];
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int mx = XC.m0 + lane; mx <= XC.m1; mx += 64) {
        const int w0 = max(0, mc * mx - 1 + J.gx), w1 = min(sx - 1, mc * mx + mc + J.gx);
        float a = INFINITY, b = -INFINITY;
        for (int x = max(w0, xs0); x <= min(w1, xs1); ++x) {
          a = fminf(a, lds_lo[x - xs0]);
          b = fmaxf(b, lds_hi[x - xs0]);
        }
        float2* p = J.partial + 2 * (((size_t)(s - 1) * J.mdy + my) * J.mdx + mx);
        if (w0 >= xs0) {
          p[0] = make_float2(a, b);
          if (w1 <= xs1) p[1] = make_float2(INFINITY, -INFINITY);
        } else {
          p[1] = make_float2(a, b);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    A = B;
    B = C;
    C.init();
    __syncthreads();
  }
}

// ranges = union of each macrocell's two partial ranges.
struct CmMerge {
  const float2* partial[kCmJobs];
  float2* ranges[kCmJobs];
  long long start[kCmJobs + 1];  // prefix sums of the macrocell counts
  int n;
};
__global__ __launch_bounds__(256) void commit_merge_kernel(CmMerge m) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.start[m.n]) return;
  int j = 0;
  while (i >= m.start[j + 1]) ++j;
  const long long c = i - m.start[j];
  const float2 a = m.partial[j][2 * c], b = m.partial[j][2 * c + 1];
  m.ranges[j][c] = make_float2(fminf(a.x, b.x), fmaxf(a.y, b.y));
}

template <typename E, int EB>
static void launch_commit_t(const McBrick* bricks, const std::vector<int>& ids, int mc, int cu_count,
                            hipStream_t st) {
  for (size_t i0 = 0; i0 < ids.size(); i0 += kCmJobs) {
    CmJobs jobs{};
    CmMerge merge{};
    int mdz_max = 1;
    for (size_t i = i0; i < std::min(ids.size(), i0 + kCmJobs); ++i) {
      const McBrick& m = bricks[ids[i]];
      const BrickG& b = m.view;
      CmJob& J = jobs.job[jobs.n];
      J.src = m.linear;
      J.dst = const_cast<void*>(b.data);
      J.partial = m.partial;
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
      J.spans = (b.sdim[0] + kCmCols - 1) / kCmCols;
      J.ygroups = (b.mdim[1] + kCmWaves - 1) / kCmWaves;
      mdz_max = std::max(mdz_max, b.mdim[2]);
      merge.partial[jobs.n] = m.partial;
      merge.ranges[jobs.n] = m.ranges;
      merge.start[jobs.n + 1] = merge.start[jobs.n] + (long long)b.mdim[0] * b.mdim[1] * b.mdim[2];
      ++jobs.n;
    }
    merge.n = jobs.n;
    // z-segment length: the fewest rounds of the chip's wave slots times a wave's
    // work (its macrocells plus the prelude and postlude rows, about 2 / mc of one)
    const double slots = (double)std::max(1, cu_count) * kCmWavesPerCu;
    int best = 1;
    double best_cost = 0.0;
    for (int seg = 1; seg <= mdz_max; ++seg) {
      double waves = 0.0;
      for (int i = 0; i < jobs.n; ++i) {
        const CmJob& J = jobs.job[i];
        waves += (double)J.spans * J.mdy * ((J.mdz + seg - 1) / seg);
      }
      const double cost = std::ceil(waves / slots) * (seg + 2.0 / mc);
      if (seg == 1 || cost < best_cost) {
        best = seg;
        best_cost = cost;
      }
    }
    long long total = 0;
    for (int i = 0; i < jobs.n; ++i) {
      CmJob& J = jobs.job[i];
      J.seg = std::min(best, J.mdz);
      J.segs = (J.mdz + J.seg - 1) / J.seg;
      J.blocks = J.ygroups * J.spans * J.segs;
      total += J.blocks;
    }
    jobs.blocks = (int)total;
    jobs.per_xcd = (int)((total + 7) / 8);
    hipLaunchKernelGGL((commit_kernel<E, cm_batch<E, EB>(), EB>), dim3((unsigned)(8 * jobs.per_xcd)), dim3(64 * kCmWaves),
                       0, st, jobs, mc);
    const long long cells = merge.start[merge.n];
    hipLaunchKernelGGL(commit_merge_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, merge);
  }
}

hipError_t launch_commit(const McBrick* bricks, int n, int mc, int cu_count, hipStream_t st) {
  std::vector<int> f32, f16p, f16h;
  for (int i = 0; i < n; ++i) (bricks[i].f16 ? (bricks[i].half16 ? f16h : f16p) : f32).push_back(i);
  if (!f32.empty()) launch_commit_t<uint32_t, 4>(bricks, f32, mc, cu_count, st);
  if (!f16p.empty()) launch_commit_t<uint16_t, 4>(bricks, f16p, mc, cu_count, st);
  if (!f16h.empty()) launch_commit_t<uint16_t, 2>(bricks, f16h, mc, cu_count, st);
  return hipGetLastError();
}

}  // namespace dpr
