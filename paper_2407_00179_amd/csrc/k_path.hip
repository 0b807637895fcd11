// Data-parallel volumetric path tracing with ray forwarding (dpr_render_path).
//
// Each brick plays one rank's part.  Rays (camera paths and their shadow rays)
// live in a pool of 64-byte records and advance in waves: in a wave a ray is
// worked on until it finishes or until its next tentative collision lies in
// another brick (it is then handed to that brick for the next wave: the
// forwarding of rays between ranks); the shadow ray a real collision spawns goes
// to the next wave while its path goes on.  Records are appended to the
// next pool with one atomic per wave.  A path's contributions land in fixed
// slots and are summed in a fixed order, so the image does not depend on the
// order of rays in the pools, nor on the bricking: the tentative collisions come
// from majorants on a grid of the whole volume and a counter-based generator
// keyed by the path.
//
// Estimator (per path): delta tracking under a piecewise-constant majorant on the
// global grid of 16^3-cell blocks (D times the TF majorant of the block's value
// range; a flight walks the blocks with a 3D DDA, so empty blocks cost nothing);
// at a real collision the throughput takes the albedo (TF colour), a shadow ray
// towards the light tracks the transmittance by ratio tracking under the same
// majorants and adds thr * light * T / 4pi; the path scatters isotropically until
// max_bounces real collisions; leaving the volume box it adds thr * env.
#include <algorithm>
#include <cmath>
#include <vector>

#include "majorant.h"
#include "march.h"
#include "runtime.hpp"

namespace dpr {

struct PRay {
  float x[3];
  float w[3];
  float t[3];     // path: throughput; shadow: weight (throughput * light / 4 pi)
  float a, b, c;  // pending path event: u1, u2, u3; shadow: T in a
  uint32_t pid;   // path id
  uint32_t e;     // path: next event index; shadow: the event that spawned it
  uint32_t meta;  // bit 31 shadow, bit 30 pending, bits 16..23 bounce (path) or slot (shadow),
                  // bits 0..15 shadow step
  int32_t brick;  // brick that works on the ray in the next wave (-1: none yet)
};
static_assert(sizeof(PRay) == 64, "ray records are 64 bytes");

constexpr uint32_t kShadowRay = 1u << 31, kPendingEvent = 1u << 30;
constexpr uint32_t kPathKey1 = 0x243F6A88u;
constexpr int kStepsPerWave = 1 << 16;  // bound on one ray's steps in one wave
constexpr int kMaxWaves = 1 << 14;
constexpr int kOwnerShift = 4;            // owner and majorant blocks of 16^3 cells
constexpr int kWavesPerCheck = 4;         // waves enqueued between reads of the pool size

struct PathG {
  const BrickG* bricks;
  int nbricks;
  // owner of each block of kOwnerCells^3 cells: a brick that holds all of it, -1
  // for a gap, -2 where bricks meet inside the block (then the bricks are searched)
  const int16_t* owner;
  int odim[3];              // blocks per axis (owner table and majorant grid)
  const float* sgrid;       // majorant per block: D * TF majorant of its value range
  float sbar;               // D * max TF opacity; only tells vacuum (0) from not
  float box[3];
  float l[3];   // unit direction towards the light
  float Ll[3];  // light radiance / (4 pi)
  float Le[3];  // environment radiance
  int B, spp;
  uint32_t seed;
  int vacuum;       // sbar == 0: nothing can collide, every path sees the environment
  float4* contrib;  // B + 1 slots per path: NEE at real collisions 0..B-1, environment at B
  PRay* out;
  int* out_count;
  int* cursor_in;   // records of the input pool taken so far (this wave)
  int* cursor_out;  // the same for the output pool: cleared for the next wave
  int out_cap;
  unsigned long long* stats;  // events, shadow steps, forwards, pool overflows, waves with rays
};

// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of two 32x32->64 products,
// the key bumped by the Weyl constants before every round but the first.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return make_uint4(c0, c1, c2, c3);
}

// ((x >> 9) + 1/2) 2^-23: exact in FP32
__device__ __forceinline__ float u01(uint32_t x) { return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f); }

__device__ __forceinline__ float exit_dist(const PathG& pg, const float x[3], const float w[3]) {
  float t = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (w[a] > 0.f)
      t = fminf(t, (pg.box[a] - x[a]) / w[a]);
    else if (w[a] < 0.f)
      t = fminf(t, -x[a] / w[a]);
  }
  return t;
}

// Brick owning the cell of point q (the hint first); -1 in a gap.
__device__ __forceinline__ int locate(const SceneG& sc, const PathG& pg, const float q[3], int hint) {
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) c[a] = min(max((int)floorf(q[a] * (float)sc.inv_h), 0), sc.dims[a] - 1);
  auto inside = [&](int i) {
    const BrickG& b = pg.bricks[i];
    return c[0] >= b.olo[0] && c[0] < b.ohi[0] && c[1] >= b.olo[1] && c[1] < b.ohi[1] && c[2] >= b.olo[2] &&
           c[2] < b.ohi[2];
  };
  if (hint >= 0 && inside(hint)) return hint;
  const int o = pg.owner[((c[2] >> kOwnerShift) * pg.odim[1] + (c[1] >> kOwnerShift)) * pg.odim[0] +
                         (c[0] >> kOwnerShift)];
  if (o != -2) return o;
  for (int i = 0; i < pg.nbricks; ++i)
    if (inside(i)) return i;
  return -1;
}

__device__ __forceinline__ float sbar_at(const SceneG& sc, const PathG& pg, const float q[3]) {
  int b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    b[a] = min(max((int)floorf(q[a] * (float)sc.inv_h), 0), sc.dims[a] - 1) >> kOwnerShift;
  return pg.sgrid[(b[2] * pg.odim[1] + b[1]) * pg.odim[0] + b[0]];
}

// Delta-tracking flight from x along w: walk the majorant blocks (3D DDA with
// per-axis next-boundary distances, advanced by one block width per step),
// accumulating majorant x length, until the sum reaches `target`; t_hit is the
// distance there.  False when the walk leaves the volume box first.
__device__ __forceinline__ bool flight(const SceneG& sc, const PathG& pg, const float x[3], const float w[3],
                                       float target, float& t_hit) {
  int b[3], step[3];
  float tmax[3], tdel[3];
  const float bw = (float)((double)(1 << kOwnerShift) * sc.h);  // block width
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    b[a] = min(max((int)floorf(x[a] * (float)sc.inv_h), 0), sc.dims[a] - 1) >> kOwnerShift;
    const float lo = (float)((double)(b[a] << kOwnerShift) * sc.h);
    const float hi = (float)((double)min((b[a] + 1) << kOwnerShift, sc.dims[a]) * sc.h);
    step[a] = w[a] > 0.f ? 1 : (w[a] < 0.f ? -1 : 0);
    tmax[a] = w[a] > 0.f ? (hi - x[a]) / w[a] : (w[a] < 0.f ? (lo - x[a]) / w[a] : INFINITY);
    tdel[a] = w[a] != 0.f ? bw / fabsf(w[a]) : INFINITY;
  }
  const float t_box = exit_dist(pg, x, w);
  float t = 0.f, acc = 0.f;
  const int max_steps = 2 * (pg.odim[0] + pg.odim[1] + pg.odim[2]) + 8;
  for (int it = 0; it < max_steps; ++it) {
    const float tn = fminf(tmax[0], fminf(tmax[1], tmax[2]));
    const float se = fminf(tn, t_box);
    const float sb = pg.sgrid[(b[2] * pg.odim[1] + b[1]) * pg.odim[0] + b[0]];
    const float gain = sb * (se - t);
    if (acc + gain >= target) {
      t_hit = t + (target - acc) / sb;
      return true;
    }
    acc += gain;
    t = se;
    if (!(se < t_box)) return false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (tmax[a] == tn) {
        b[a] = min(max(b[a] + step[a], 0), pg.odim[a] - 1);
        tmax[a] += tdel[a];
      }
    }
  }
  return false;
}

// Extinction and albedo at q from brick b (trilinear sample, TF lookup).
template <typename T, bool WIDE>
__device__ __forceinline__ void medium(const SceneG& sc, const BrickG& b, const float4* __restrict__ tfb,
                                       const float4* __restrict__ tfs, const float q[3], float& sigma,
                                       float alb[3]) {
  int64_t p[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) p[a] = __double2ll_rn(((double)q[a] * sc.inv_h - 0.5) * kFix);
  Gather<T> g;
  gather<T, WIDE>(sc, b, p, g);
  const float v = trilerp(g);
  float x = (v - sc.tf_lo) * sc.tf_scale;
  x = fminf(fmaxf(x, 0.f), (float)(sc.ntf - 1));
  const int j = min((int)x, sc.ntf - 2);
  const float w = x - (float)j;
  const float4 tb = tfb[j], ts = tfs[j];
  sigma = sc.density * fmaf(w, ts.w, tb.w);
  alb[0] = fmaf(w, ts.x, tb.x);
  alb[1] = fmaf(w, ts.y, tb.y);
  alb[2] = fmaf(w, ts.z, tb.z);
}

__device__ __forceinline__ void add_contrib(const PathG& pg, uint32_t pid, int slot, float r, float g, float b) {
  pg.contrib[(size_t)pid * (pg.B + 1) + slot] = make_float4(r, g, b, 0.f);
}

// Append up to two records per lane with one atomic per wave (called by every
// lane of the wave at the same point).
__device__ __forceinline__ void emit2(const PathG& pg, const PRay& ra, bool ha, const PRay& rb, bool hb) {
  const int lane = threadIdx.x & 63;
  const uint64_t ma = __ballot(ha), mb = __ballot(hb);
  const int na = __popcll(ma), total = na + __popcll(mb);
  if (total == 0) return;
  int base = 0;
  if (lane == 0) base = atomicAdd(pg.out_count, total);
  base = __shfl(base, 0);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int ia = base + __popcll(ma & lt), ib = base + na + __popcll(mb & lt);
  bool over = false;
  if (ha) {
    if (ia < pg.out_cap) pg.out[ia] = ra;
    else over = true;
  }
  if (hb) {
    if (ib < pg.out_cap) pg.out[ib] = rb;
    else over = true;
  }
  if (over) atomicAdd(pg.stats + 3, 1ull);
}

__device__ __forceinline__ void wave_stats(const PathG& pg, unsigned ev, unsigned st, unsigned fw) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ev += __shfl_xor(ev, o);
    st += __shfl_xor(st, o);
    fw += __shfl_xor(fw, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (ev) atomicAdd(pg.stats + 0, (unsigned long long)ev);
    if (st) atomicAdd(pg.stats + 1, (unsigned long long)st);
    if (fw) atomicAdd(pg.stats + 2, (unsigned long long)fw);
  }
}

// Camera paths: one per (pixel, sample), started at the volume box entry with no
// brick.  The first flight needs only the majorant grid, which every rank holds,
// so the brick of the first tentative collision starts the path without a
// hand-over.
__global__ __launch_bounds__(256) void path_init_kernel(PathG pg, CamG cam, int W, int H) {
  const long long total = (long long)W * H * pg.spp;
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  PRay r{};
  bool live = false;
  if (id < total) {
    const uint32_t pid = (uint32_t)id;
    const int pix = (int)(id / pg.spp);
    double d[3];
    camera_ray(cam, pix % W, pix / W, d);
    const double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {pg.box[0], pg.box[1], pg.box[2]};
    double t_in, t_out;
    if (!pg.vacuum && clip_box(cam.eye, d, lo, hi, t_in, t_out)) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        r.x[a] = (float)(cam.eye[a] + t_in * d[a]);
        r.w[a] = (float)d[a];
        r.t[a] = 1.f;
      }
      r.pid = pid;
      r.brick = -1;
      live = true;
    } else {
      add_contrib(pg, pid, pg.B, pg.Le[0], pg.Le[1], pg.Le[2]);
    }
  }
  const PRay none{};
  emit2(pg, r, live, none, false);
}

// n_in: device count of the input pool (written by the previous wave).  A resident
// grid takes its records through pg.cursor_in; the loop runs while any lane of the
// wave holds a ray, so the refills and appends stay convergent.
template <typename T, bool WIDE>
__global__ __launch_bounds__(256) void path_trace_kernel(SceneG sc, PathG pg, const float4* __restrict__ tf,
                                                         const PRay* __restrict__ in,
                                                         const int* __restrict__ n_in_dev) {
  extern __shared__ float4 tf_lds[];
  float4* tfb = tf_lds;
  float4* tfs = tf_lds + sc.ntf;
  stage_tf(tf, sc.ntf, tfb, tfs, threadIdx.x, 256);
  __syncthreads();
  const int n_in = min(*n_in_dev, pg.out_cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (n_in > 0) atomicAdd(pg.stats + 4, 1ull);
    *pg.cursor_out = 0;
  }
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  unsigned ev = 0, st = 0, fw = 0;
  // Each lane holds one ray.  Idle lanes take the next records of the input pool
  // (one atomic per wave); a camera path stays in its lane across real collisions
  // (its shadow ray goes to the next wave), so the wave's long chains overlap.
  PRay r{};
  bool have = false, exhausted = false;
  for (;;) {
    const uint64_t idle = __ballot(!have);
    if (idle && !exhausted) {
      int base = 0;
      if (lane == 0) base = atomicAdd(pg.cursor_in, __popcll(idle));
      base = __shfl(base, 0);
      if (base + __popcll(idle) >= n_in) exhausted = true;
      if (!have) {
        const int i = base + __popcll(idle & lt_mask);
        if (i < n_in) {
          r = in[i];
          have = true;
        }
      }
    }
    if (__ballot(have) == 0) break;
  PRay ra{}, rb{};
  bool ha = false, hb = false;
  if (have) {
    have = false;
    if (r.meta & kShadowRay) {
      const int slot = (int)((r.meta >> 16) & 0xff);
      for (int it = 0;; ++it) {
        if (it == kStepsPerWave) {  // keep it for the next wave
          ra = r;
          ha = true;
          break;
        }
        if (!(r.meta & kPendingEvent)) {
          const uint4 q = philox(r.pid, r.e, 1u, r.meta & 0xffffu, pg.seed, kPathKey1);
          float s;
          ++st;
          if (!flight(sc, pg, r.x, r.w, -logf(u01(q.x)), s)) {
            add_contrib(pg, r.pid, slot, r.t[0] * r.a, r.t[1] * r.a, r.t[2] * r.a);
            break;
          }
#pragma unroll
          for (int a = 0; a < 3; ++a) r.x[a] = fmaf(s, r.w[a], r.x[a]);
          r.meta |= kPendingEvent;
        }
        const int owner = locate(sc, pg, r.x, r.brick);
        if (owner >= 0 && owner != r.brick) {
          r.brick = owner;
          ra = r;
          ha = true;
          ++fw;
          break;
        }
        float sigma = 0.f, alb[3];
        if (owner >= 0) medium<T, WIDE>(sc, pg.bricks[owner], tfb, tfs, r.x, sigma, alb);
        const float sbq = sbar_at(sc, pg, r.x);
        if (sbq > 0.f) r.a *= 1.f - sigma / sbq;
        r.meta = (r.meta & ~(kPendingEvent | 0xffffu)) | (((r.meta & 0xffffu) + 1u) & 0xffffu);
        if (r.a == 0.f) break;  // nothing more can reach the light (the slot stays 0)
      }
    } else {
      for (int it = 0;; ++it) {
        if (it == kStepsPerWave) {
          ra = r;
          ha = true;
          break;
        }
        if (!(r.meta & kPendingEvent)) {
          const uint4 q = philox(r.pid, r.e, 0u, 0u, pg.seed, kPathKey1);
          float t;
          if (!flight(sc, pg, r.x, r.w, -logf(u01(q.x)), t)) {  // leaves the volume
            add_contrib(pg, r.pid, pg.B, r.t[0] * pg.Le[0], r.t[1] * pg.Le[1], r.t[2] * pg.Le[2]);
            break;
          }
#pragma unroll
          for (int a = 0; a < 3; ++a) r.x[a] = fmaf(t, r.w[a], r.x[a]);
          r.a = u01(q.y);
          r.b = u01(q.z);
          r.c = u01(q.w);
          r.meta |= kPendingEvent;
        }
        const int owner = locate(sc, pg, r.x, r.brick);
        if (owner >= 0 && owner != r.brick) {
          if (r.brick >= 0) {
            r.brick = owner;
            ra = r;
            ha = true;
            ++fw;
            break;
          }
          r.brick = owner;  // a camera path starts with the brick of its first tentative collision
        }
        ++ev;
        float sigma = 0.f, alb[3] = {0.f, 0.f, 0.f};
        if (owner >= 0) medium<T, WIDE>(sc, pg.bricks[owner], tfb, tfs, r.x, sigma, alb);
        r.meta &= ~kPendingEvent;
        const uint32_t e = r.e++;
        const float sbq = sbar_at(sc, pg, r.x);
        if (sbq > 0.f && r.a < sigma / sbq) {  // real collision
          const int k = (int)((r.meta >> 16) & 0xff);
#pragma unroll
          for (int a = 0; a < 3; ++a) r.t[a] *= alb[a];
          PRay s{};
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            s.x[a] = r.x[a];
            s.w[a] = pg.l[a];
            s.t[a] = r.t[a] * pg.Ll[a];
          }
          s.a = 1.f;
          s.pid = r.pid;
          s.e = e;
          s.meta = kShadowRay | ((uint32_t)k << 16);
          s.brick = owner;
          rb = s;
          hb = true;
          if (k + 1 >= pg.B) break;  // the path ends at its last real collision
          r.meta = (r.meta & ~(0xffu << 16)) | ((uint32_t)(k + 1) << 16);
          const float z = 1.f - 2.f * r.b;
          const float rr = sqrtf(fmaxf(0.f, 1.f - z * z));
          float sp, cp;
          sincosf(6.28318530717958647692f * r.c, &sp, &cp);
          r.w[0] = rr * cp;
          r.w[1] = rr * sp;
          r.w[2] = z;
          have = true;  // the path goes on in this lane
          break;
        }
      }
    }
  }
  emit2(pg, ra, ha, rb, hb);
  }
  wave_stats(pg, ev, st, fw);
}

// Pixel radiance: the contributions of its paths, summed in slot order, then
// averaged over its samples.
__global__ __launch_bounds__(256) void path_resolve_kernel(PathG pg, int n_pixels, float4* __restrict__ out_rgba,
                                                           float* __restrict__ out_depth) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n_pixels) return;
  float sr = 0.f, sg = 0.f, sb = 0.f;
  for (int s = 0; s < pg.spp; ++s) {
    const float4* c = pg.contrib + ((size_t)p * pg.spp + s) * (pg.B + 1);
    float lr = 0.f, lg = 0.f, lb = 0.f;
    for (int k = 0; k <= pg.B; ++k) {
      const float4 v = c[k];
      lr += v.x;
      lg += v.y;
      lb += v.z;
    }
    sr += lr;
    sg += lg;
    sb += lb;
  }
  const float inv = 1.f / (float)pg.spp;
  out_rgba[p] = make_float4(sr * inv, sg * inv, sb * inv, 1.f);
  out_depth[p] = INFINITY;
}

// ---- majorant grid: value range and TF majorant per 16^3-cell block of the
// global grid, over voxels [16 k - 1, 16 k + 16] per axis.  Every brick reduces
// its owned voxels in each block window it meets; the ranges meet through
// order-preserving integer atomics (so the grid does not depend on the bricking).
__device__ __forceinline__ uint32_t ord_of(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_of(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

struct BlkRangeJob {
  const void* vox;  // linear stored copy, x fastest
  int s0[3];        // global voxel of stored element 0
  int sdim[3];
  int olo[3], ohi[3];  // owned voxels [olo, ohi)
  int k0[3], kn[3];    // blocks whose window meets the owned voxels
  int odim[3];
};

template <typename T>
__global__ __launch_bounds__(256) void block_range_kernel(BlkRangeJob J, uint32_t* __restrict__ lo_enc,
                                                          uint32_t* __restrict__ hi_enc) {
  __shared__ float red[2][4];
  const int bid = blockIdx.x;
  const int k[3] = {J.k0[0] + bid % J.kn[0], J.k0[1] + (bid / J.kn[0]) % J.kn[1],
                    J.k0[2] + bid / (J.kn[0] * J.kn[1])};
  int a0[3], n[3];
  bool empty = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    a0[a] = max((k[a] << kOwnerShift) - 1, J.olo[a]);
    const int a1 = min((k[a] << kOwnerShift) + (1 << kOwnerShift), J.ohi[a] - 1);
    n[a] = a1 - a0[a] + 1;
    empty |= n[a] <= 0;
  }
  if (empty) return;  // uniform over the workgroup
  const T* vox = (const T*)J.vox;
  float mn = INFINITY, mx = -INFINITY;
  const int total = n[0] * n[1] * n[2];
  for (int i = threadIdx.x; i < total; i += 256) {
    const int x = a0[0] + i % n[0], y = a0[1] + (i / n[0]) % n[1], z = a0[2] + i / (n[0] * n[1]);
    const size_t off = ((size_t)(z - J.s0[2]) * J.sdim[1] + (y - J.s0[1])) * J.sdim[0] + (x - J.s0[0]);
    float v;
    if constexpr (sizeof(T) == 2)
      v = __half2float(vox[off]);
    else
      v = vox[off];
    mn = fminf(mn, v);
    mx = fmaxf(mx, v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, o));
    mx = fmaxf(mx, __shfl_xor(mx, o));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = mn;
    red[1][threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int wv = 1; wv < 4; ++wv) {
      mn = fminf(mn, red[0][wv]);
      mx = fmaxf(mx, red[1][wv]);
    }
    const size_t idx = ((size_t)k[2] * J.odim[1] + k[1]) * J.odim[0] + k[0];
    atomicMin(lo_enc + idx, ord_of(mn));
    atomicMax(hi_enc + idx, ord_of(mx));
  }
}

__global__ __launch_bounds__(256) void block_majorant_kernel(const uint32_t* __restrict__ lo_enc,
                                                             const uint32_t* __restrict__ hi_enc, int n,
                                                             const float4* __restrict__ tf, int ntf, float tf_lo,
                                                             float tf_hi, float density, float* __restrict__ sgrid) {
  __shared__ float alpha[kMaxTF];
  for (int i = threadIdx.x; i < ntf; i += 256) alpha[i] = tf[i].w;
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t lo = lo_enc[i];
  float m = 0.f;  // a block no brick reached (a gap) is empty
  if (lo != 0xffffffffu) m = tf_majorant(make_float2(float_of(lo), float_of(hi_enc[i])), alpha, ntf, tf_lo, tf_hi);
  sgrid[i] = density * m;
}

struct PathState {
  PRay* pool[2] = {nullptr, nullptr};
  size_t cap = 0;  // records per pool
  float4* contrib = nullptr;
  size_t contrib_cap = 0;
  BrickG* d_bricks = nullptr;
  int brick_cap = 0;
  int16_t* d_owner = nullptr;
  size_t owner_cap = 0;
  uint32_t* d_lo = nullptr;  // encoded block ranges
  uint32_t* d_hi = nullptr;
  float* d_sgrid = nullptr;
  size_t grid_cap = 0;
  uint64_t grid_commit = ~0ull, grid_tf = ~0ull;
  size_t grid_n = 0;
  uint64_t owner_version = 0;
  int odim[3] = {0, 0, 0};
  int* d_count = nullptr;  // [0], [1]: sizes of the two pools
  unsigned long long* d_stats = nullptr;
  int* h_count = nullptr;  // pinned
};

void path_state_free(PathState* p) {
  if (!p) return;
  dev_free(p->pool[0]);
  dev_free(p->pool[1]);
  dev_free(p->contrib);
  dev_free(p->d_bricks);
  dev_free(p->d_owner);
  dev_free(p->d_lo);
  dev_free(p->d_hi);
  dev_free(p->d_sgrid);
  dev_free(p->d_count);
  dev_free(p->d_stats);
  host_free(p->h_count);
  delete p;
}

template <typename T, bool WIDE>
static void launch_trace(const SceneG& sc, const PathG& pg, const float4* tf, const PRay* in, const int* n,
                         int grid, size_t lds, hipStream_t st) {
  // (pg.cursor_in counts the records of `in` taken; pg.cursor_out is cleared by the kernel)
  hipLaunchKernelGGL((path_trace_kernel<T, WIDE>), dim3((unsigned)grid), dim3(256), lds, st, sc, pg, tf, in, n);
}

}  // namespace dpr

using namespace dpr;

extern "C" dpr_status dpr_render_path(dpr_world w, const dpr_path_params* prm, dpr_frame out,
                                      dpr_path_stats* stats) {
  if (!w || !prm || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_path: NULL argument");
  if (!w->committed) return fail(DPR_ERR_INVALID_STATE, "dpr_render_path: world not committed");
  if (!w->tf_set) return fail(DPR_ERR_INVALID_STATE, "dpr_render_path: no transfer function set");
  if (!w->cam_set) return fail(DPR_ERR_INVALID_STATE, "dpr_render_path: no camera set");
  if (out->dev != w->dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_path: frame of another device");
  if (out->w != w->cam.width || out->h != w->cam.height)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_path: frame %dx%d != camera %dx%d", out->w, out->h,
                w->cam.width, w->cam.height);
  if (prm->max_bounces < 1 || prm->max_bounces > 255)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_path: max_bounces %d outside [1, 255]", prm->max_bounces);
  if (prm->spp < 1) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_path: spp %d", prm->spp);
  double ln = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(prm->light_dir[a]) || !(prm->light_rgb[a] >= 0.f) || !std::isfinite(prm->light_rgb[a]) ||
        !(prm->env_rgb[a] >= 0.f) || !std::isfinite(prm->env_rgb[a]))
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_path: light or environment not finite and >= 0");
    ln += (double)prm->light_dir[a] * prm->light_dir[a];
  }
  if (!(ln > 0.0)) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_path: light_dir is zero");
  const int K = (int)w->bricks.size();
  for (const auto& b : w->bricks)
    if (b.dtype != w->bricks[0].dtype)
      return fail(DPR_ERR_UNSUPPORTED, "dpr_render_path: bricks of different element types");
  const long long n_paths = (long long)out->w * out->h * prm->spp;
  const int B = prm->max_bounces;
  const long long slots = n_paths * (B + 1);
  if (n_paths > 0x7fffffffll || slots > 0x7fffffffll)
    return fail(DPR_ERR_UNSUPPORTED, "dpr_render_path: %lld paths x %d slots exceed 2^31", n_paths, B + 1);
  hipStream_t st = w->dev->stream;
  if (!w->path) w->path = new PathState;
  PathState* ps = w->path;
  dpr_status s;
  if ((size_t)slots > ps->cap) {
    DPR_HIP(hipStreamSynchronize(st));
    dev_free(ps->pool[0]);
    dev_free(ps->pool[1]);
    ps->pool[0] = ps->pool[1] = nullptr;
    ps->cap = 0;
    if ((s = dev_alloc((void**)&ps->pool[0], (size_t)slots * sizeof(PRay), "path ray pool")) != DPR_OK) return s;
    if ((s = dev_alloc((void**)&ps->pool[1], (size_t)slots * sizeof(PRay), "path ray pool")) != DPR_OK) return s;
    ps->cap = (size_t)slots;
  }
  if ((size_t)slots > ps->contrib_cap) {
    DPR_HIP(hipStreamSynchronize(st));
    dev_free(ps->contrib);
    ps->contrib = nullptr;
    ps->contrib_cap = 0;
    if ((s = dev_alloc((void**)&ps->contrib, (size_t)slots * sizeof(float4), "path contributions")) != DPR_OK)
      return s;
    ps->contrib_cap = (size_t)slots;
  }
  if (K > ps->brick_cap) {
    DPR_HIP(hipStreamSynchronize(st));
    dev_free(ps->d_bricks);
    ps->d_bricks = nullptr;
    if ((s = dev_alloc((void**)&ps->d_bricks, (size_t)K * sizeof(BrickG), "path bricks")) != DPR_OK) return s;
    ps->brick_cap = K;
  }
  if (!ps->d_count) {
    if ((s = dev_alloc((void**)&ps->d_count, 4 * sizeof(int), "path pool sizes and cursors")) != DPR_OK) return s;
    if ((s = dev_alloc((void**)&ps->d_stats, 5 * sizeof(unsigned long long), "path stats")) != DPR_OK) return s;
    if ((s = host_alloc((void**)&ps->h_count, 2 * sizeof(int), "path pool sizes (host)")) != DPR_OK) return s;
  }
  // owner table of 16^3-cell blocks, rebuilt when bricks were added
  int od[3];
  for (int a = 0; a < 3; ++a) od[a] = (int)((w->dims[a] + (1 << kOwnerShift) - 1) >> kOwnerShift);
  const size_t n_own = (size_t)od[0] * od[1] * od[2];
  if (ps->owner_version != w->geo_version || ps->odim[0] != od[0] || ps->odim[1] != od[1] || ps->odim[2] != od[2]) {
    std::vector<int16_t> own(n_own);
    for (int bz = 0; bz < od[2]; ++bz)
      for (int by = 0; by < od[1]; ++by)
        for (int bx = 0; bx < od[0]; ++bx) {
          const int64_t lo[3] = {(int64_t)bx << kOwnerShift, (int64_t)by << kOwnerShift, (int64_t)bz << kOwnerShift};
          int64_t hi[3];
          for (int a = 0; a < 3; ++a) hi[a] = std::min(lo[a] + (1 << kOwnerShift), w->dims[a]);
          int found = -1, overlaps = 0;
          bool whole = false;
          for (int i = 0; i < K; ++i) {
            const auto& b = w->bricks[i];
            bool ov = true, con = true;
            for (int a = 0; a < 3; ++a) {
              ov &= b.olo[a] < hi[a] && lo[a] < b.ohi[a];
              con &= b.olo[a] <= lo[a] && hi[a] <= b.ohi[a];
            }
            if (ov) {
              ++overlaps;
              found = i;
              whole = con;
            }
          }
          own[((size_t)bz * od[1] + by) * od[0] + bx] =
              (int16_t)(overlaps == 0 ? -1 : (overlaps == 1 && whole ? found : -2));
        }
    if (n_own > ps->owner_cap) {
      DPR_HIP(hipStreamSynchronize(st));
      dev_free(ps->d_owner);
      ps->d_owner = nullptr;
      ps->owner_cap = 0;
      if ((s = dev_alloc((void**)&ps->d_owner, n_own * sizeof(int16_t), "path owner table")) != DPR_OK) return s;
      ps->owner_cap = n_own;
    }
    DPR_HIP(hipMemcpyAsync(ps->d_owner, own.data(), n_own * sizeof(int16_t), hipMemcpyHostToDevice, st));
    DPR_HIP(hipStreamSynchronize(st));
    for (int a = 0; a < 3; ++a) ps->odim[a] = od[a];
    ps->owner_version = w->geo_version;
  }
  std::vector<BrickG> views(K);
  bool wide = false;
  for (int i = 0; i < K; ++i) {
    views[i] = w->bricks[i].device_view(false, w->params.flags & DPR_FLAG_WIDE_OFFSETS);
    wide |= views[i].wide;
  }
  // the views are staged through pageable memory: wait for the copy before they change
  DPR_HIP(hipMemcpyAsync(ps->d_bricks, views.data(), (size_t)K * sizeof(BrickG), hipMemcpyHostToDevice, st));

  const SceneG sc = make_scene(w);
  float amax = 0.f;
  // the majorant: D times the largest TF opacity (the TF is staged on the host)
  {
    std::vector<float4> tfh(w->ntf);
    DPR_HIP(hipMemcpyAsync(tfh.data(), w->tf_dev, (size_t)w->ntf * sizeof(float4), hipMemcpyDeviceToHost, st));
    DPR_HIP(hipStreamSynchronize(st));
    for (const auto& v : tfh) amax = std::max(amax, v.w);
  }
  // majorant grid, rebuilt after a commit or a TF change
  if (ps->grid_commit != w->commit_version || ps->grid_tf != w->tf_version || ps->grid_n != n_own) {
    if (n_own > ps->grid_cap) {
      DPR_HIP(hipStreamSynchronize(st));
      dev_free(ps->d_lo);
      dev_free(ps->d_hi);
      dev_free(ps->d_sgrid);
      ps->d_lo = ps->d_hi = nullptr;
      ps->d_sgrid = nullptr;
      ps->grid_cap = 0;
      if ((s = dev_alloc((void**)&ps->d_lo, n_own * sizeof(uint32_t), "block ranges")) != DPR_OK) return s;
      if ((s = dev_alloc((void**)&ps->d_hi, n_own * sizeof(uint32_t), "block ranges")) != DPR_OK) return s;
      if ((s = dev_alloc((void**)&ps->d_sgrid, n_own * sizeof(float), "block majorants")) != DPR_OK) return s;
      ps->grid_cap = n_own;
    }
    DPR_HIP(hipMemsetAsync(ps->d_lo, 0xff, n_own * sizeof(uint32_t), st));
    DPR_HIP(hipMemsetAsync(ps->d_hi, 0, n_own * sizeof(uint32_t), st));
    for (const auto& b : w->bricks)
      if (!b.linear)
        return fail(DPR_ERR_INVALID_STATE,
                    "dpr_render_path: the block majorants need the bricks' linear copies, which were released");
    for (const auto& b : w->bricks) {
      BlkRangeJob J{};
      J.vox = b.linear;
      int blocks = 1;
      for (int a = 0; a < 3; ++a) {
        J.s0[a] = (int)(b.olo[a] - b.glo[a]);
        J.sdim[a] = b.sdim[a];
        J.olo[a] = (int)b.olo[a];
        J.ohi[a] = (int)b.ohi[a];
        // window [16 k - 1, 16 k + 16] meets [olo, ohi - 1]
        const int k0 = J.olo[a] >= 16 ? (J.olo[a] - 16 + 15) / 16 : 0;
        const int k1 = std::min(J.ohi[a] / 16, od[a] - 1);
        J.k0[a] = k0;
        J.kn[a] = std::max(0, k1 - k0 + 1);
        J.odim[a] = od[a];
        blocks *= J.kn[a];
      }
      if (blocks == 0) continue;
      if (b.dtype == DPR_F16)
        hipLaunchKernelGGL(block_range_kernel<__half>, dim3((unsigned)blocks), dim3(256), 0, st, J, ps->d_lo,
                           ps->d_hi);
      else
        hipLaunchKernelGGL(block_range_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, J, ps->d_lo,
                           ps->d_hi);
      DPR_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(block_majorant_kernel, dim3((unsigned)((n_own + 255) / 256)), dim3(256), 0, st, ps->d_lo,
                       ps->d_hi, (int)n_own, w->tf_dev, w->ntf, w->tf_lo, w->tf_hi, w->density, ps->d_sgrid);
    DPR_HIP(hipGetLastError());
    ps->grid_commit = w->commit_version;
    ps->grid_tf = w->tf_version;
    ps->grid_n = n_own;
  }

  PathG pg{};
  pg.bricks = ps->d_bricks;
  pg.sgrid = ps->d_sgrid;
  pg.nbricks = K;
  pg.owner = ps->d_owner;
  for (int a = 0; a < 3; ++a) pg.odim[a] = od[a];
  pg.sbar = sc.density * amax;
  for (int a = 0; a < 3; ++a) pg.box[a] = (float)((double)w->dims[a] * sc.h);
  const double inv_l = 1.0 / std::sqrt(ln);
  const float inv4pi = (float)(1.0 / (4.0 * M_PI));
  for (int a = 0; a < 3; ++a) {
    pg.l[a] = (float)(-(double)prm->light_dir[a] * inv_l);
    pg.Ll[a] = prm->light_rgb[a] * inv4pi;
    pg.Le[a] = prm->env_rgb[a];
  }
  pg.B = B;
  pg.spp = prm->spp;
  pg.seed = prm->seed;
  pg.contrib = ps->contrib;
  pg.out_count = ps->d_count;
  pg.out_cap = (int)ps->cap;
  pg.stats = ps->d_stats;
  DPR_HIP(hipMemsetAsync(ps->contrib, 0, (size_t)slots * sizeof(float4), st));
  DPR_HIP(hipMemsetAsync(ps->d_count, 0, 4 * sizeof(int), st));
  DPR_HIP(hipMemsetAsync(ps->d_stats, 0, 5 * sizeof(unsigned long long), st));

  int cur = 0;
  pg.out = ps->pool[cur];
  pg.vacuum = !(pg.sbar > 0.f);
  const CamG cam = make_cam(w->cam);
  hipLaunchKernelGGL(path_init_kernel, dim3((unsigned)((n_paths + 255) / 256)), dim3(256), 0, st, pg, cam, out->w,
                     out->h);
  DPR_HIP(hipGetLastError());
  DPR_HIP(hipMemcpyAsync(ps->h_count, ps->d_count, sizeof(int), hipMemcpyDeviceToHost, st));
  DPR_HIP(hipStreamSynchronize(st));
  int n = ps->h_count[0];
  const size_t lds = 2 * sizeof(float4) * (size_t)sc.ntf;
  const bool f16 = K > 0 && w->bricks[0].dtype == DPR_F16;
  // a resident grid walks whatever the previous wave left; the host reads the pool
  // size only every kWavesPerCheck waves (later waves of a batch may find it empty)
  const void* fn = f16 ? (wide ? (const void*)path_trace_kernel<__half, true> : (const void*)path_trace_kernel<__half, false>)
                       : (wide ? (const void*)path_trace_kernel<float, true> : (const void*)path_trace_kernel<float, false>);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  const int grid = w->dev->cu_count * per_cu;
  int enqueued = 0;
  while (n > 0) {
    for (int j = 0; j < kWavesPerCheck; ++j) {
      if (++enqueued > kMaxWaves) return fail(DPR_ERR_DEVICE, "dpr_render_path: more than %d waves", kMaxWaves);
      const PRay* in = ps->pool[cur];
      const int* n_in = ps->d_count + cur;
      cur ^= 1;
      pg.cursor_in = ps->d_count + 2 + (cur ^ 1);
      pg.out = ps->pool[cur];
      pg.out_count = ps->d_count + cur;
      pg.cursor_out = ps->d_count + 2 + cur;
      DPR_HIP(hipMemsetAsync(pg.out_count, 0, sizeof(int), st));
      if (f16)
        wide ? launch_trace<__half, true>(sc, pg, w->tf_dev, in, n_in, grid, lds, st)
             : launch_trace<__half, false>(sc, pg, w->tf_dev, in, n_in, grid, lds, st);
      else
        wide ? launch_trace<float, true>(sc, pg, w->tf_dev, in, n_in, grid, lds, st)
             : launch_trace<float, false>(sc, pg, w->tf_dev, in, n_in, grid, lds, st);
      DPR_HIP(hipGetLastError());
    }
    DPR_HIP(hipMemcpyAsync(ps->h_count, ps->d_count + cur, sizeof(int), hipMemcpyDeviceToHost, st));
    DPR_HIP(hipStreamSynchronize(st));
    n = ps->h_count[0];
    if ((size_t)n > ps->cap) return fail(DPR_ERR_DEVICE, "dpr_render_path: ray pool overflow (%d > %zu)", n, ps->cap);
  }
  const int P = out->w * out->h;
  hipLaunchKernelGGL(path_resolve_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, pg, P,
                     (float4*)out->rgba, out->depth);
  DPR_HIP(hipGetLastError());
  unsigned long long hs[5] = {0, 0, 0, 0, 0};
  DPR_HIP(hipMemcpyAsync(hs, ps->d_stats, sizeof(hs), hipMemcpyDeviceToHost, st));
  DPR_HIP(hipStreamSynchronize(st));
  if (hs[3]) return fail(DPR_ERR_DEVICE, "dpr_render_path: %llu rays did not fit the pool", hs[3]);
  if (stats) {
    stats->paths = n_paths;
    stats->events = (int64_t)hs[0];
    stats->shadow_steps = (int64_t)hs[1];
    stats->forwards = (int64_t)hs[2];
    stats->waves = (int32_t)hs[4];
  }
  return DPR_OK;
}
