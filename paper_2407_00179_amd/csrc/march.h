// Resumable per-ray emission-absorption march through one brick.
//
// Sample points advance in exact 32.32 fixed point (global voxel-centre units),
// so the point of segment s is the same integer whichever way the ray got there:
// in one call, in budgeted slices (persistent kernel), with or without skipping.
// The lattice is walked in runs of consecutive segments whose sample points share
// one macrocell; the run length is computed exactly in integers, a run in a
// macrocell of majorant 0 is skipped in O(1), and the other runs sample every
// segment with no per-sample macrocell logic.  Voxel gathers of the next sample
// are issued before the current sample is shaded.  For bricks below 4 GiB a voxel
// address is a 32-bit byte offset from the brick base.
//
// Iso-surfaces (ISO): the sides (v >= v_iso) of consecutive samples are compared
// at every lattice point the brick owns (those in [t_in, t_out)); the first change
// of side is an opaque surface, lit at the linearly interpolated crossing with the
// gradient of the trilinear patch there, and closes the ray.  A macrocell is then
// skipped only when its majorant is 0, its value range lies on one side of v_iso,
// and that side is the previous sample's (classes encoded in the majorant: 0 below,
// -1 at or above, positive: sample it).
#pragma once

#include "device_common.h"

namespace dpr {

constexpr double kFix = 4294967296.0;  // 2^32
constexpr int kShadeRun = 4;            // samples per run in a non-empty macrocell (even)

struct RayState {
  int64_t p[3];          // sample point of segment s, 32.32 fixed point (global voxel-centre coords)
  int64_t dp[3];         // advance per segment
  double t_in, t_out;    // clipped parametric range (world units)
  double tau;            // optical depth accumulated so far
  int s, s0, s1;         // next segment, first and last segment
  int n;                 // logical samples processed
  float dl_first, dl_last;  // D * clipped length of the first / last segment
  float T, cr, cg, cb;   // transmittance and premultiplied colour
  float pv;              // iso-surfaces: value of the previous sample
  int pst;               // iso-surfaces: bit 0 side of the previous sample, bit 1 the next
                         // sample closes a tested pair, bit 2 pv holds the value
};

constexpr int kIsoSide = 1, kIsoPair = 2, kIsoKnown = 4;

// Clip the ray against the brick's owned box and set up its march.  Returns false
// on a miss (zero-length chords included).
__device__ __forceinline__ bool ray_begin(const SceneG& sc, const BrickG& b, const double o[3], const double d[3],
                                          RayState& r) {
  double lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = b.olo[a] * sc.h;
    hi[a] = b.ohi[a] * sc.h;
  }
  if (!clip_box(o, d, lo, hi, r.t_in, r.t_out)) return false;
  const double dt = sc.dt;
  int s0 = (int)floor(r.t_in / dt);
  int s1 = (int)ceil(r.t_out / dt) - 1;
  // lengths of the clipped end segments; a non-positive one is dropped
  double lf = fmin((s0 + 1) * dt, r.t_out) - fmax(s0 * dt, r.t_in);
  if (!(lf > 0.0)) {
    ++s0;
    lf = fmin((s0 + 1) * dt, r.t_out) - fmax(s0 * dt, r.t_in);
  }
  double ll = fmin((s1 + 1) * dt, r.t_out) - fmax(s1 * dt, r.t_in);
  if (!(ll > 0.0)) {
    --s1;
    ll = fmin((s1 + 1) * dt, r.t_out) - fmax(s1 * dt, r.t_in);
  }
  // (s1 < s0 only through rounding at a vanishing chord: a hit with no samples)
  r.s = r.s0 = s0;
  r.s1 = s1;
  r.dl_first = sc.density * (float)lf;
  r.dl_last = sc.density * (float)ll;
  const double tm = (s0 + 0.5) * dt;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double dv = d[a] * sc.inv_h;
    const double g = fma(tm, dv, o[a] * sc.inv_h - 0.5);
    r.p[a] = __double2ll_rn(g * kFix);
    r.dp[a] = __double2ll_rn(dt * dv * kFix);
  }
  r.tau = 0.0;
  r.n = 0;
  r.T = 1.f;
  r.cr = r.cg = r.cb = 0.f;
  return true;
}

// Largest j >= 0 with p + j*dp inside [b_lo, b_hi) on one axis (the current point
// is inside).  Exact: floating-point quotient corrected in integers.
__device__ __forceinline__ int steps_inside(int64_t p, int64_t dp, int64_t b_lo, int64_t b_hi, int cap) {
  int64_t num, den;
  if (dp > 0) {
    if (b_hi == INT64_MAX) return cap;
    num = b_hi - 1 - p;
    den = dp;
  } else if (dp < 0) {
    if (b_lo == INT64_MIN) return cap;
    num = p - b_lo;
    den = -dp;
  } else {
    return cap;
  }
  int64_t q = (int64_t)((double)num / (double)den);
  if (q * den > num) --q;
  else if ((q + 1) * den <= num) ++q;
  return q < (int64_t)cap ? (int)q : cap;
}

// Voxel index (stored, relative to the brick) and fraction along one axis of a
// 32.32 fixed-point sample point, clamped to the global domain [0, n - 1].
__device__ __forceinline__ int axis_index(int64_t p, int n, int slo, int sdim) {
  const int hi = (int)(p >> 32);
  const int i0 = min(max(hi, 0), n - 2);
  // commit guarantees i0 - slo lies in [0, sdim - 2]; the clamp only guards memory
  return min(max(i0 - slo, 0), sdim - 2);
}
__device__ __forceinline__ float axis_frac(int64_t p, int n) {
  const int hi = (int)(p >> 32);
  const float fr = (float)(uint32_t)(p & 0xffffffffll) * (1.0f / 4294967296.0f);
  return (hi < 0) ? 0.f : ((hi > n - 2) ? 1.f : fr);
}

template <typename T>
struct Gather {
  float v[8];
  float fx, fy, fz;
};

// The loaded voxels of a sample's 8-voxel footprint, before decoding (FP16: the
// four voxel pairs as loaded), so a request in flight holds as few registers as
// possible.
template <typename T>
struct Voxels;
template <>
struct Voxels<float> {
  float v[8];
};
template <>
struct Voxels<__half> {
  uint32_t c[4];
};

// Load the 8 voxels around a sample point.  Byte offsets from the brick base:
// 32-bit sums of per-axis terms for bricks below 4 GiB; WIDE (the blocked array is
// 4 GiB or more, or 64-bit offsets were asked for): 32-bit element indices (a
// brick holds fewer than 2^32 elements), widened and scaled once per load.
// Either way the loads are global loads.  An FP16 brick is stored as voxel pairs
// when addressed with 32-bit offsets and as 2-byte voxels when addressed with
// 64-bit offsets (the commit picks the layout and the addressing together).
template <typename T, bool WIDE>
__device__ __forceinline__ void load_voxels(const SceneG& sc, const BrickG& b, const int64_t p[3], Voxels<T>& g) {
  const int lx = axis_index(p[0], sc.dims[0], b.slo[0], b.sdim[0]);
  const int ly = axis_index(p[1], sc.dims[1], b.slo[1], b.sdim[1]);
  const int lz = axis_index(p[2], sc.dims[2], b.slo[2], b.sdim[2]);
  using GC = const char __attribute__((address_space(1)))*;
  if constexpr (sizeof(T) == 4) {
    constexpr int SH = 2;
    uint32_t x0, x1, y0, y1, z0, z1;
    if constexpr (WIDE) {
      x0 = blk_x(lx), x1 = blk_x(lx + 1);
      y0 = blk_y(ly, b.bsy), y1 = blk_y(ly + 1, b.bsy);
      z0 = blk_z(lz, b.bsz), z1 = blk_z(lz + 1, b.bsz);
    } else {
      const uint32_t bsy = b.bsy << SH, bsz = b.bsz << SH;
      x0 = blkb_x<SH>(lx), x1 = blkb_x<SH>(lx + 1);
      y0 = blkb_y<SH>(ly, bsy), y1 = blkb_y<SH>(ly + 1, bsy);
      z0 = blkb_z<SH>(lz, bsz), z1 = blkb_z<SH>(lz + 1, bsz);
    }
    // byte offset of the element at the sum of the per-axis terms
    auto off = [](uint32_t e) {
      if constexpr (WIDE)
        return (uint64_t)e << SH;
      else
        return e;
    };
    const uint32_t a00 = x0 + y0, a01 = x0 + y1;
    // voxel lx + 1 follows voxel lx in memory unless lx ends a 4-voxel x-run, so
    // each x-pair is one 8-byte load; lanes at a run's end read lx + 1 on their
    // own.
    const float2 c0 = load_pair_f32(b.data, off(a00 + z0)), c1 = load_pair_f32(b.data, off(a01 + z0));
    const float2 c2 = load_pair_f32(b.data, off(a00 + z1)), c3 = load_pair_f32(b.data, off(a01 + z1));
    g.v[0] = c0.x;
    g.v[1] = c0.y;
    g.v[2] = c1.x;
    g.v[3] = c1.y;
    g.v[4] = c2.x;
    g.v[5] = c2.y;
    g.v[6] = c3.x;
    g.v[7] = c3.y;
    if ((lx & 3) == 3) {
      const uint32_t a10 = x1 + y0, a11 = x1 + y1;
      g.v[1] = load_voxel_b<T>(b.data, off(a10 + z0));
      g.v[3] = load_voxel_b<T>(b.data, off(a11 + z0));
      g.v[5] = load_voxel_b<T>(b.data, off(a10 + z1));
      g.v[7] = load_voxel_b<T>(b.data, off(a11 + z1));
    }
  } else if constexpr (WIDE) {
    // FP16 voxels (2 bytes: the layout of bricks addressed with 64-bit offsets):
    // the aligned 4-voxel run holding lx is one 8-byte load and the pair
    // (lx, lx + 1) is shifted out of it; lanes whose lx ends a run read lx + 1 on
    // their own.  Element offsets are 32-bit sums (a brick holds fewer than 2^32
    // elements), widened and scaled once per load.
    using GU64 = const uint64_t __attribute__((address_space(1)))*;
    using GU16 = const uint16_t __attribute__((address_space(1)))*;
    const uint32_t y0 = blk_y(ly, b.bsy), y1 = blk_y(ly + 1, b.bsy);
    const uint32_t z0 = blk_z(lz, b.bsz), z1 = blk_z(lz + 1, b.bsz);
    const uint32_t x0 = blk_x(lx & ~3);
    auto off = [](uint32_t e) { return (uint64_t)e << 1; };
    const uint32_t a00 = x0 + y0, a01 = x0 + y1;
    const uint32_t rs = (uint32_t)(lx & 3) << 4;
    g.c[0] = (uint32_t)(*(GU64)((GC)b.data + off(a00 + z0)) >> rs);
    g.c[1] = (uint32_t)(*(GU64)((GC)b.data + off(a01 + z0)) >> rs);
    g.c[2] = (uint32_t)(*(GU64)((GC)b.data + off(a00 + z1)) >> rs);
    g.c[3] = (uint32_t)(*(GU64)((GC)b.data + off(a01 + z1)) >> rs);
    if ((lx & 3) == 3) {
      const uint32_t x1 = blk_x(lx + 1), a10 = x1 + y0, a11 = x1 + y1;
      g.c[0] = (g.c[0] & 0xffffu) | ((uint32_t) * (GU16)((GC)b.data + off(a10 + z0)) << 16);
      g.c[1] = (g.c[1] & 0xffffu) | ((uint32_t) * (GU16)((GC)b.data + off(a11 + z0)) << 16);
      g.c[2] = (g.c[2] & 0xffffu) | ((uint32_t) * (GU16)((GC)b.data + off(a10 + z1)) << 16);
      g.c[3] = (g.c[3] & 0xffffu) | ((uint32_t) * (GU16)((GC)b.data + off(a11 + z1)) << 16);
    }
  } else {
    // FP16 voxel pairs (4 bytes, the layout of bricks below 4 GiB): each element
    // holds the voxels (x, x + 1), one aligned 4-byte load per pair
    constexpr int SH = 2;
    using GU = const uint32_t __attribute__((address_space(1)))*;
    const uint32_t bsy = b.bsy << SH, bsz = b.bsz << SH;
    const uint32_t x0 = blkb_x<SH>(lx);
    const uint32_t y0 = blkb_y<SH>(ly, bsy), y1 = blkb_y<SH>(ly + 1, bsy);
    const uint32_t z0 = blkb_z<SH>(lz, bsz), z1 = blkb_z<SH>(lz + 1, bsz);
    const uint32_t a00 = x0 + y0, a01 = x0 + y1;
    g.c[0] = *(GU)((GC)b.data + a00 + z0);
    g.c[1] = *(GU)((GC)b.data + a01 + z0);
    g.c[2] = *(GU)((GC)b.data + a00 + z1);
    g.c[3] = *(GU)((GC)b.data + a01 + z1);
  }
}

// The 8 footprint voxels as FP32: (x0, x1) at (y0, z0), (y1, z0), (y0, z1), (y1, z1).
template <typename T>
__device__ __forceinline__ void decode_voxels(const Voxels<T>& g, float v[8]) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = g.v[k];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float2 c = unpack_pair_f16(g.c[k]);
      v[2 * k] = c.x;
      v[2 * k + 1] = c.y;
    }
  }
}

// Trilinear fractions of a sample point.
__device__ __forceinline__ void sample_frac(const SceneG& sc, const int64_t p[3], float& fx, float& fy, float& fz) {
  fx = axis_frac(p[0], sc.dims[0]);
  fy = axis_frac(p[1], sc.dims[1]);
  fz = axis_frac(p[2], sc.dims[2]);
}

// Gather the 8 voxels around a sample point and its trilinear fractions.
template <typename T, bool WIDE>
__device__ __forceinline__ void gather(const SceneG& sc, const BrickG& b, const int64_t p[3], Gather<T>& g) {
  sample_frac(sc, p, g.fx, g.fy, g.fz);
  Voxels<T> raw;
  load_voxels<T, WIDE>(sc, b, p, raw);
  decode_voxels<T>(raw, g.v);
}

template <typename T>
__device__ __forceinline__ float trilerp(const Gather<T>& g) {
  const float c00 = fmaf(g.fx, g.v[1] - g.v[0], g.v[0]), c01 = fmaf(g.fx, g.v[3] - g.v[2], g.v[2]);
  const float c10 = fmaf(g.fx, g.v[5] - g.v[4], g.v[4]), c11 = fmaf(g.fx, g.v[7] - g.v[6], g.v[6]);
  const float c0 = fmaf(g.fy, c01 - c00, c00), c1 = fmaf(g.fy, c11 - c10, c10);
  return fmaf(g.fz, c1 - c0, c0);
}

// Shade one sample of value v; returns true when the ray terminates early.
__device__ __forceinline__ bool shade_v(const SceneG& sc, const float4* __restrict__ tfb,
                                        const float4* __restrict__ tfs, float v, float Dl, double& tau_acc,
                                        float& tr, float& cr, float& cg, float& cb) {
  float x = (v - sc.tf_lo) * sc.tf_scale;
  x = fminf(fmaxf(x, 0.f), (float)(sc.ntf - 1));
  const int j = min((int)x, sc.ntf - 2);
  const float w = x - (float)j;
  const float4 tb = tfb[j], ts = tfs[j];
  const float A = fmaf(w, ts.w, tb.w);
  const float tau = Dl * A;
  if (tau > 0.f) {
    tau_acc += (double)tau;
    const float tn = __expf(-(float)tau_acc);
    const float wgt = tr - tn;
    cr = fmaf(wgt, fmaf(w, ts.x, tb.x), cr);
    cg = fmaf(wgt, fmaf(w, ts.y, tb.y), cg);
    cb = fmaf(wgt, fmaf(w, ts.z, tb.z), cb);
    tr = tn;
    return 1.f - tr >= sc.ert;
  }
  return false;
}

template <typename T>
__device__ __forceinline__ bool shade(const SceneG& sc, const float4* __restrict__ tfb,
                                      const float4* __restrict__ tfs, const Gather<T>& g, float Dl, double& tau_acc,
                                      float& tr, float& cr, float& cg, float& cb) {
  return shade_v(sc, tfb, tfs, trilerp(g), Dl, tau_acc, tr, cr, cg, cb);
}

// Set up the ray (ray_begin) and, for iso-surfaces, the pair at the brick entry:
// when the first processed segment starts exactly at t_in its lattice point is
// this brick's, and the sample half a step before the entry opens the pair.
template <typename T, bool WIDE, bool ISO>
__device__ __forceinline__ bool ray_start(const SceneG& sc, const BrickG& b, const double o[3], const double d[3],
                                          RayState& r) {
  if (!ray_begin(sc, b, o, d, r)) return false;
  if constexpr (ISO) {
    r.pv = 0.f;
    r.pst = 0;
    if ((double)r.s0 * sc.dt >= r.t_in) {
      const int64_t q[3] = {r.p[0] - r.dp[0], r.p[1] - r.dp[1], r.p[2] - r.dp[2]};
      Gather<T> g;
      gather<T, WIDE>(sc, b, q, g);
      r.pv = trilerp(g);
      r.pst = kIsoPair | kIsoKnown | (r.pv >= sc.iso ? kIsoSide : 0);
    }
  }
  return true;
}

// The opaque surface between samples s - 1 and s (value vs; q: the fixed-point
// point of sample s): crossing by linear interpolation, normal = gradient of the
// trilinear patch there, colour = TF colour at v_iso * (k_a + k_d |cos|).
template <typename T, bool WIDE>
__device__ __forceinline__ void iso_hit(const SceneG& sc, const BrickG& b, const float4* __restrict__ tfb,
                                     const float4* __restrict__ tfs, const int64_t q[3], const int64_t dq[3],
                                     float vs, int pst, float pv, float& tr, float& cr, float& cg, float& cb) {
  const int64_t qp[3] = {q[0] - dq[0], q[1] - dq[1], q[2] - dq[2]};
  float vp = pv;
  if (!(pst & kIsoKnown)) {  // the previous sample was skipped: its value now
    Gather<T> g;
    gather<T, WIDE>(sc, b, qp, g);
    vp = trilerp(g);
  }
  const float f = (sc.iso - vp) / (vs - vp);
  int64_t qh[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) qh[a] = qp[a] + __double2ll_rn((double)f * (double)dq[a]);
  Gather<T> g;
  gather<T, WIDE>(sc, b, qh, g);
  const float* v = g.v;
  // d/dx, d/dy, d/dz of the patch: the edge differences, interpolated in the other two axes
  const float x0 = fmaf(g.fy, (v[3] - v[2]) - (v[1] - v[0]), v[1] - v[0]);
  const float x1 = fmaf(g.fy, (v[7] - v[6]) - (v[5] - v[4]), v[5] - v[4]);
  const float gx = fmaf(g.fz, x1 - x0, x0);
  const float y0 = fmaf(g.fx, (v[3] - v[1]) - (v[2] - v[0]), v[2] - v[0]);
  const float y1 = fmaf(g.fx, (v[7] - v[5]) - (v[6] - v[4]), v[6] - v[4]);
  const float gy = fmaf(g.fz, y1 - y0, y0);
  const float z0 = fmaf(g.fx, (v[5] - v[1]) - (v[4] - v[0]), v[4] - v[0]);
  const float z1 = fmaf(g.fx, (v[7] - v[3]) - (v[6] - v[2]), v[6] - v[2]);
  const float gz = fmaf(g.fy, z1 - z0, z0);
  // the ray direction is parallel to the per-segment advance.  Every product and
  // sum is spelled out (fmaf, __fmul_rn): left to contraction, the compiler may
  // associate these sums differently in different kernels, and the skip and
  // no-skip marches would then differ in the last bit
  const float dx = (float)dq[0], dy = (float)dq[1], dz = (float)dq[2];
  const float nn = fmaf(gz, gz, fmaf(gy, gy, __fmul_rn(gx, gx)));
  const float dd = fmaf(dz, dz, fmaf(dy, dy, __fmul_rn(dx, dx)));
  const float dot = fmaf(gz, dz, fmaf(gy, dy, __fmul_rn(gx, dx)));
  const float cosv = nn > 0.f ? fabsf(dot) / sqrtf(__fmul_rn(nn, dd)) : 1.f;
  float x = (sc.iso - sc.tf_lo) * sc.tf_scale;
  x = fminf(fmaxf(x, 0.f), (float)(sc.ntf - 1));
  const int j = min((int)x, sc.ntf - 2);
  const float w = x - (float)j;
  const float4 tb = tfb[j], ts = tfs[j];
  const float lit = fmaf(sc.iso_kd, fminf(cosv, 1.f), sc.iso_ka);
  cr = fmaf(tr, __fmul_rn(fmaf(w, ts.x, tb.x), lit), cr);
  cg = fmaf(tr, __fmul_rn(fmaf(w, ts.y, tb.y), lit), cg);
  cb = fmaf(tr, __fmul_rn(fmaf(w, ts.z, tb.z), lit), cb);
  tr = 0.f;
}

// Emission-absorption march (no iso-surface) with a deeper pipeline: the voxels
// of the next two samples are in flight while a sample is shaded, and the
// majorant of the next run's macrocell is requested at the start of a run, so a
// lane waits on memory about once per sample rather than once per sample plus
// once per run.  Three gather buffers rotate; a run of a multiple of three
// samples leaves the two buffers after it holding the next run's first two
// samples.  Same lattice points, the same skip decisions, the same shading
// order and the same termination test as the single-lookahead loop, so the
// same bits.
constexpr int kPipeRun = 6;  // samples per run in a non-empty macrocell (a multiple of 3)

template <typename T, bool SKIP, bool WIDE>
__device__ __forceinline__ bool ray_advance_ea(const SceneG& sc, const BrickG& b, const float4* __restrict__ tfb,
                                               const float4* __restrict__ tfs, RayState& r, int budget,
                                               int min_lanes) {
  const float Ddt = sc.density * sc.dt_f;
  const int64_t half = 0x80000000ll;
  int s = r.s;
  int n = r.n;
  int64_t p0 = r.p[0], p1 = r.p[1], p2 = r.p[2];
  const int64_t d0 = r.dp[0], d1 = r.dp[1], d2 = r.dp[2];
  float tr = r.T, cr = r.cr, cg = r.cg, cb = r.cb;
  double tau_acc = r.tau;
  bool done = false;
  Voxels<T> ga, gb, gc;
  bool pre = false;      // ga, gb hold the voxels of samples s and s + 1
  int64_t q0 = 0, q1 = 0, q2 = 0;  // point of the next sample to request
  float mj_next = 0.f;
  bool have_mj = false;  // mj_next is the majorant of sample s's macrocell
  auto macrocell = [&](int64_t x, int64_t y, int64_t z, int m[3]) {
    const int64_t pp[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int cell = (int)((pp[a] + half) >> 32);
      m[a] = min(max((cell - b.olo[a]) >> b.mc_shift, 0), b.mdim[a] - 1);
    }
  };
  auto majorant = [&](const int m[3]) { return ld_global(b.majorant, (m[2] * b.mdim[1] + m[1]) * b.mdim[0] + m[0]); };
  auto request = [&](Voxels<T>& g) {
    const int64_t q[3] = {q0, q1, q2};
    load_voxels<T, WIDE>(sc, b, q, g);
    q0 += d0;
    q1 += d1;
    q2 += d2;
  };
  // shade sample s from its voxels; its fractions come from its point, p
  auto step = [&](const Voxels<T>& g) -> bool {
    Gather<T> gg;
    const int64_t pc[3] = {p0, p1, p2};
    sample_frac(sc, pc, gg.fx, gg.fy, gg.fz);
    decode_voxels<T>(g, gg.v);
    const float Dl = (s == r.s0) ? r.dl_first : ((s == r.s1) ? r.dl_last : Ddt);
    ++n;
    ++s;
    p0 += d0;
    p1 += d1;
    p2 += d2;
    return shade<T>(sc, tfb, tfs, gg, Dl, tau_acc, tr, cr, cg, cb);
  };
  while (!done && s <= r.s1 && budget > 0) {
    // at a run boundary: return early (unfinished) once fewer than min_lanes lanes
    // of the wave are still marching, so the caller can refill the idle ones
    if (__popcll(__ballot(1)) < min_lanes) break;
    int run = min(r.s1 - s + 1, budget);
    if constexpr (SKIP) {
      int m[3];
      macrocell(p0, p1, p2, m);
      const float mj = have_mj ? mj_next : majorant(m);
      if (mj == 0.f) {
        // exactly the samples left inside this empty macrocell (outer cells
        // unbounded); every one has opacity exactly 0
        const int64_t pp[3] = {p0, p1, p2}, dd[3] = {d0, d1, d2};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int ma = m[a];
          const int64_t blo = (ma == 0) ? INT64_MIN
                                        : ((int64_t)(b.olo[a] + (ma << b.mc_shift)) << 32) - half;
          const int64_t bhi = (ma == b.mdim[a] - 1) ? INT64_MAX
                                                    : ((int64_t)(b.olo[a] + ((ma + 1) << b.mc_shift)) << 32) - half;
          run = min(run, 1 + steps_inside(pp[a], dd[a], blo, bhi, run - 1));
        }
        s += run;
        n += run;
        budget -= run;
        p0 += (int64_t)run * d0;
        p1 += (int64_t)run * d1;
        p2 += (int64_t)run * d2;
        pre = false;
        have_mj = false;
        continue;
      }
      // a non-empty macrocell: a fixed number of samples, then look again (the
      // run may cross into other macrocells; a sample of zero opacity changes
      // nothing, so its length needs no exact boundary arithmetic)
      run = min(run, kPipeRun);
      int mn[3];
      macrocell(p0 + (int64_t)run * d0, p1 + (int64_t)run * d1, p2 + (int64_t)run * d2, mn);
      mj_next = majorant(mn);
      have_mj = true;
    }
    budget -= run;
    if (!pre) {
      q0 = p0;
      q1 = p1;
      q2 = p2;
      request(ga);
      request(gb);
    }
    // the request two samples ahead is unconditional (past the run's last sample
    // it reads clamped, in-brick voxels that are never used).  Three buffers
    // rotate by position (no register copies: copying a buffer whose load is in
    // flight would wait for it), and the loop body has no exit: a step past the
    // run's end or after termination is skipped, not left, which keeps the
    // control flow simple enough for the buffers to stay in place
    for (int i = 0; i < run; i += 3) {
      request(gc);
      if (!done) done = step(ga);
      request(ga);
      if (!done && i + 1 < run) done = step(gb);
      request(gb);
      if (!done && i + 2 < run) done = step(gc);
    }
    pre = !done && run % 3 == 0;
  }
  // the fixed-point position always corresponds to segment s
  r.s = s;
  r.p[0] = p0;
  r.p[1] = p1;
  r.p[2] = p2;
  r.T = tr;
  r.cr = cr;
  r.cg = cg;
  r.cb = cb;
  r.tau = tau_acc;
  r.n = n;
  return done || s > r.s1;
}

// Advance by at most `budget` lattice segments.  Returns true once the ray is
// finished: past its last segment, or terminated early (1 - T >= ert, tested
// after every segment that changed T).
template <typename T, bool SKIP, bool WIDE, bool ISO>
__device__ __forceinline__ bool ray_advance(const SceneG& sc, const BrickG& b, const float4* __restrict__ tfb,
                                            const float4* __restrict__ tfs, RayState& r, int budget,
                                            int min_lanes = 0) {
  if constexpr (!ISO) return ray_advance_ea<T, SKIP, WIDE>(sc, b, tfb, tfs, r, budget, min_lanes);
  const float Ddt = sc.density * sc.dt_f;
  int s = r.s;
  int n = r.n;
  int64_t p0 = r.p[0], p1 = r.p[1], p2 = r.p[2];
  const int64_t d0 = r.dp[0], d1 = r.dp[1], d2 = r.dp[2];
  float tr = r.T, cr = r.cr, cg = r.cg, cb = r.cb;
  double tau_acc = r.tau;
  bool done = false;
  int pst = ISO ? r.pst : 0;
  float pv = ISO ? r.pv : 0.f, vh = 0.f;
  bool hit = false;
  // ga holds the voxels of the current sample point when pre is set: a run of even
  // length ends with the next sample's gather in ga, and the next run reuses it
  Gather<T> ga, gb;
  bool pre = false;
  while (!done && s <= r.s1 && budget > 0) {
    // at a run boundary: return early (unfinished) once fewer than min_lanes lanes
    // of the wave are still marching, so the caller can refill the idle ones
    if (__popcll(__ballot(1)) < min_lanes) break;
    int run = min(r.s1 - s + 1, budget);
    bool empty = false;
    if (SKIP) {
      // macrocell of the current sample point: cell = floor(g + 1/2)
      const int64_t half = 0x80000000ll;
      const int64_t pp[3] = {p0, p1, p2};
      int m[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int cell = (int)((pp[a] + half) >> 32);
        m[a] = min(max((cell - b.olo[a]) >> b.mc_shift, 0), b.mdim[a] - 1);
      }
      const float mj = ld_global(b.majorant, (m[2] * b.mdim[1] + m[1]) * b.mdim[0] + m[0]);
      if constexpr (ISO) {
        empty = mj <= 0.f && (!(pst & kIsoPair) || ((mj < 0.f) == (bool)(pst & kIsoSide)));
        if (empty) pst = kIsoPair | (mj < 0.f ? kIsoSide : 0);
      } else {
        empty = mj == 0.f;
      }
      if (empty) {
        // exactly the samples left inside this empty macrocell (outer cells unbounded)
        const int64_t dd[3] = {d0, d1, d2};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int ma = m[a];
          const int64_t blo = (ma == 0) ? INT64_MIN
                                        : ((int64_t)(b.olo[a] + (ma << b.mc_shift)) << 32) - half;
          const int64_t bhi = (ma == b.mdim[a] - 1) ? INT64_MAX
                                                    : ((int64_t)(b.olo[a] + ((ma + 1) << b.mc_shift)) << 32) - half;
          run = min(run, 1 + steps_inside(pp[a], dd[a], blo, bhi, run - 1));
        }
      } else {
        // a non-empty macrocell: a fixed number of samples, then look again.  The
        // run may cross into other macrocells; shading is correct everywhere (a
        // sample of zero opacity changes nothing), so its length needs no exact
        // boundary arithmetic and the lanes of a wave stay in step
        run = min(run, kShadeRun);
      }
    }
    if (empty) {  // every sample in the run has opacity exactly 0
      s += run;
      n += run;
      budget -= run;
      p0 += (int64_t)run * d0;
      p1 += (int64_t)run * d1;
      p2 += (int64_t)run * d2;
      pre = false;
      continue;
    }
    budget -= run;
    // one sample per step, the next sample's voxels requested before this one is
    // shaded; two steps per trip alternate the gather buffers (no register copies).
    // The request is unconditional (past the run's last sample it reads clamped,
    // in-brick voxels that are never used), so the wait before shading covers only
    // the older request.
    auto step = [&](const Gather<T>& g) -> bool {
      const float Dl = (s == r.s0) ? r.dl_first : ((s == r.s1) ? r.dl_last : Ddt);
      ++n;
      ++s;
      if constexpr (ISO) {
        const float v = trilerp(g);
        const int side = v >= sc.iso ? kIsoSide : 0;
        if ((pst & kIsoPair) && side != (pst & kIsoSide)) {  // the surface: no emission from this segment
          hit = true;
          vh = v;
          return true;
        }
        pst = kIsoPair | kIsoKnown | side;
        pv = v;
        return shade_v(sc, tfb, tfs, v, Dl, tau_acc, tr, cr, cg, cb);
      } else {
        return shade<T>(sc, tfb, tfs, g, Dl, tau_acc, tr, cr, cg, cb);
      }
    };
    if (!pre) {
      const int64_t pc[3] = {p0, p1, p2};
      gather<T, WIDE>(sc, b, pc, ga);
    }
    for (int i = 0;;) {
      p0 += d0;
      p1 += d1;
      p2 += d2;
      {
        const int64_t pn[3] = {p0, p1, p2};
        gather<T, WIDE>(sc, b, pn, gb);
      }
      if (step(ga)) {
        done = true;
        break;
      }
      if (++i >= run) break;
      p0 += d0;
      p1 += d1;
      p2 += d2;
      {
        const int64_t pn[3] = {p0, p1, p2};
        gather<T, WIDE>(sc, b, pn, ga);
      }
      if (step(gb)) {
        done = true;
        break;
      }
      if (++i >= run) break;
    }
    pre = (run & 1) == 0;
  }
  if constexpr (ISO) {
    if (hit) {  // the hit sample is s - 1, one segment behind the current point
      const int64_t q[3] = {p0 - d0, p1 - d1, p2 - d2};
      const int64_t dq[3] = {d0, d1, d2};
      iso_hit<T, WIDE>(sc, b, tfb, tfs, q, dq, vh, pst, pv, tr, cr, cg, cb);
    }
  }
  // the fixed-point position always corresponds to segment s
  r.s = s;
  r.p[0] = p0;
  r.p[1] = p1;
  r.p[2] = p2;
  r.T = tr;
  r.cr = cr;
  r.cg = cg;
  r.cb = cb;
  r.tau = tau_acc;
  r.n = n;
  if constexpr (ISO) {
    r.pst = pst;
    r.pv = pv;
  }
  return done || s > r.s1;
}

// Stage the TF as (entry, next - entry) pairs so a lookup is one FMA per channel.
__device__ __forceinline__ void stage_tf(const float4* __restrict__ tf, int ntf, float4* base, float4* slope,
                                         int tid, int nthreads) {
  for (int i = tid; i < ntf; i += nthreads) {
    float4 a = tf[i];
    float4 b = (i + 1 < ntf) ? tf[i + 1] : a;
    base[i] = a;
    slope[i] = make_float4(b.x - a.x, b.y - a.y, b.z - a.z, b.w - a.w);
  }
}

}  // namespace dpr
