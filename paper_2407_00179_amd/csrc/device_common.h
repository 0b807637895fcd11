// Device-side data structures and helpers shared by the HIP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace dpr {

constexpr int kBlockEdge = 8;         // bricks are stored as 8^3-voxel blocks
// FP16 bricks are stored in one of two layouts, chosen per world at commit:
// 4-byte elements holding the voxel pair (x, x + 1) -- one load per trilinear
// x-pair, the faster layout while gathers mostly hit the cache -- or 2-byte
// elements holding one voxel -- half the bytes, so half the cache lines per
// sample and half the memory -- once a brick's pair copy would reach 4 GiB.  The
// 2-byte layout always goes with 64-bit voxel offsets, so the kernels' WIDE
// variants read it and their narrow variants read pairs.
constexpr uint64_t kF16HalvesFrom = 1ull << 32;  // pair-copy bytes from which FP16 bricks store halves
constexpr int kBlockVoxels = 512;
constexpr int kMaxTF = 1024;          // transfer-function entries held in LDS

// Pinhole camera in FP64: ray d = normalize(f + x r + y u) with
// x = (2(px+.5)/W - 1) sx and y = (1 - 2(py+.5)/H) sy.
struct CamG {
  double eye[3];
  double f[3], r[3], u[3];
  double sx, sy;
  int W, H;
};

// One brick as the kernels see it.
struct BrickG {
  const void* data;       // 8^3-blocked voxels (interleaved order inside a block, blocks x-fastest)
  int slo[3];             // global voxel index of stored voxel (0,0,0)
  int sdim[3];            // stored dims
  uint32_t bsy, bsz;      // element stride of one block row in y / one block slab in z
  int olo[3], ohi[3];     // owned global cells [olo, ohi)
  const float* majorant;  // per macrocell, x fastest (may be null when skipping is off)
  int mdim[3];            // macrocell grid
  int mc_shift;           // log2(macrocell edge)
  int wide;               // 64-bit voxel offsets (blocked array of 4 GiB or more, an FP16 brick
                          // stored as 2-byte voxels, or asked for); else 32-bit byte offsets
};

// Scene-wide render constants.
struct SceneG {
  int dims[3];            // global dims
  double h, inv_h, dt;
  float dt_f, density, ert, tf_lo, tf_scale;  // tf_scale = (N-1)/(hi-lo)
  int ntf;
  // opaque iso-surface (iso_on): value, ambient and diffuse weights
  int iso_on;
  float iso, iso_ka, iso_kd;
};

// Inside an 8^3 block the 9 bits of a voxel's index interleave its coordinates:
// bits 0-1 x&3, bit 2 y&1, bit 3 z&1, bit 4 (y>>1)&1, bit 5 (z>>1)&1, bit 6
// (x>>2)&1, bit 7 (y>>2)&1, bit 8 (z>>2)&1.  Every 16 consecutive voxels form a
// 4x2x2 brick, every 32 a 4x4x2 one and every 64 a 4x4x4 one, so the 8 voxels
// around a sample span fewer cache lines than with whole x rows, whatever the
// ray's direction; the index stays a sum of one term per axis.
__device__ __forceinline__ uint32_t blk_x(int i) {
  return ((uint32_t)(i >> 3) << 9) + (uint32_t)(i & 3) + ((uint32_t)(i & 4) << 4);
}
__device__ __forceinline__ uint32_t blk_y(int j, uint32_t bsy) {
  return (uint32_t)(j >> 3) * bsy + ((uint32_t)(j & 1) << 2) + ((uint32_t)(j & 2) << 3) + ((uint32_t)(j & 4) << 5);
}
__device__ __forceinline__ uint32_t blk_z(int k, uint32_t bsz) {
  return (uint32_t)(k >> 3) * bsz + ((uint32_t)(k & 1) << 3) + ((uint32_t)(k & 2) << 4) + ((uint32_t)(k & 4) << 6);
}

// Byte offsets of the same layout for elements of 1 << SH bytes (bsy_b, bsz_b:
// byte strides), for bricks whose blocked array is below 4 GiB: a voxel is then
// one global load from the brick's base (a scalar register pair) plus a 32-bit
// vector offset, with no per-lane 64-bit address arithmetic.
template <int SH>
__device__ __forceinline__ uint32_t blkb_x(int i) {
  return ((uint32_t)(i >> 3) << (9 + SH)) + (blk_x(i & 7) << SH);
}
template <int SH>
__device__ __forceinline__ uint32_t blkb_y(int j, uint32_t bsy_b) {
  return (uint32_t)(j >> 3) * bsy_b + (blk_y(j & 7, 0u) << SH);
}
template <int SH>
__device__ __forceinline__ uint32_t blkb_z(int k, uint32_t bsz_b) {
  return (uint32_t)(k >> 3) * bsz_b + (blk_z(k & 7, 0u) << SH);
}
template <typename T, typename Off>
__device__ __forceinline__ float load_voxel_b(const void* base, Off boff) {
  using GC = const char __attribute__((address_space(1)))*;
  const GC q = (GC)base + boff;
  if constexpr (sizeof(T) == 2)
    return __half2float(__ushort_as_half(*(const unsigned short __attribute__((address_space(1)))*)q));
  else
    return *(const float __attribute__((address_space(1)))*)q;
}

// An F32 voxel at byte offset boff and the element after it in memory, in one
// load aligned to 4 bytes only.  A blocked array carries kPairSlack spare bytes so
// the element after its last voxel can be read.  Off: uint32_t byte offsets for
// blocked arrays below 4 GiB, uint64_t above; the pointer is in the global address
// space either way, so the load is a global (not flat) load and waits only on the
// vector-memory counter.
constexpr size_t kPairSlack = 64;
template <typename Off>
__device__ __forceinline__ float2 load_pair_f32(const void* base, Off boff) {
  typedef float F2 __attribute__((ext_vector_type(2), aligned(4)));
  using GC = const char __attribute__((address_space(1)))*;
  const F2 f = *(const F2 __attribute__((address_space(1)))*)((GC)base + boff);
  return make_float2(f.x, f.y);
}

// An FP16 brick's element: the halves of voxel x (low) and voxel x + 1 (high).
__device__ __forceinline__ float2 unpack_pair_f16(uint32_t u) {
  return make_float2(__half2float(__ushort_as_half((unsigned short)(u & 0xffffu))),
                     __half2float(__ushort_as_half((unsigned short)(u >> 16))));
}
template <typename Off>
__device__ __forceinline__ float2 load_pair_f16(const void* base, Off boff) {
  using GC = const char __attribute__((address_space(1)))*;
  return unpack_pair_f16(*(const uint32_t __attribute__((address_space(1)))*)((GC)base + boff));
}

// Element i of an array in device memory, read with a global (not flat) load:
// pointers fetched from memory lose their address space, and a flat load also
// holds back the LDS counter that transfer-function lookups wait on.
template <typename T>
__device__ __forceinline__ T ld_global(const T* p, size_t i) {
  return ((const T __attribute__((address_space(1)))*)p)[i];
}

// Ray through pixel (px, py); returns the unit direction.
__device__ __forceinline__ void camera_ray(const CamG& c, int px, int py, double d[3]) {
  double x = (2.0 * (px + 0.5) / c.W - 1.0) * c.sx;
  double y = (1.0 - 2.0 * (py + 0.5) / c.H) * c.sy;
  double v0 = c.f[0] + x * c.r[0] + y * c.u[0];
  double v1 = c.f[1] + x * c.r[1] + y * c.u[1];
  double v2 = c.f[2] + x * c.r[2] + y * c.u[2];
  double inv = 1.0 / sqrt(v0 * v0 + v1 * v1 + v2 * v2);
  d[0] = v0 * inv;
  d[1] = v1 * inv;
  d[2] = v2 * inv;
}

// Slab test against the box [lo, hi]; t_in = max(t_near, 0), hit iff t_out > t_in.
__device__ __forceinline__ bool clip_box(const double o[3], const double d[3], const double lo[3],
                                         const double hi[3], double& t_in, double& t_out) {
  double tn = -INFINITY, tf = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < lo[a] || o[a] > hi[a]) return false;
      continue;
    }
    double t0 = (lo[a] - o[a]) / d[a];
    double t1 = (hi[a] - o[a]) / d[a];
    tn = fmax(tn, fmin(t0, t1));
    tf = fmin(tf, fmax(t0, t1));
  }
  t_in = fmax(tn, 0.0);
  t_out = tf;
  return t_out > t_in;
}

}  // namespace dpr
