// Brick ingest (8^3 relayout), macrocell ranges, transfer-function majorants and
// the per-brick emission-absorption ray march, for gfx950.
#include "device_common.h"
#include "kernels.h"

namespace dpr {

// ------------------------------------------------------------------ relayout
// Linear x-fastest stored brick -> 8^3 blocks (x fastest inside a block, blocks
// x-fastest).  One thread per output element; padding voxels are zero and are
// never read by the sampler.
template <typename E>
__global__ __launch_bounds__(256) void relayout_kernel(const E* __restrict__ src, E* __restrict__ dst, int sx,
                                                       int sy, int sz, int bx, int by, uint64_t total) {
  uint64_t idx = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  uint32_t w = (uint32_t)(idx & 511);
  uint64_t blk = idx >> 9;
  int x = (int)(blk % (uint64_t)bx) * 8 + (int)(w & 7);
  uint64_t r = blk / (uint64_t)bx;
  int y = (int)(r % (uint64_t)by) * 8 + (int)((w >> 3) & 7);
  int z = (int)(r / (uint64_t)by) * 8 + (int)(w >> 6);
  E v = E(0);
  if (x < sx && y < sy && z < sz) v = src[((uint64_t)z * sy + y) * sx + x];
  dst[idx] = v;
}

// ------------------------------------------------------------------ macrocell ranges
// One workgroup per macrocell: min/max over owned-relative voxels [mc m - 1, mc m + mc]
// per axis, clipped to the stored range (stored index = owned index + ghost_lo).
template <typename T>
__global__ __launch_bounds__(256) void macrocell_kernel(const T* __restrict__ vox, int sx, int sy, int sz,
                                                        uint32_t bsy, uint32_t bsz, int gx, int gy, int gz,
                                                        int mc, int mdx, int mdy, int mdz,
                                                        float2* __restrict__ ranges) {
  int m = blockIdx.x;
  int mx = m % mdx, my = (m / mdx) % mdy, mz = m / (mdx * mdy);
  int x0 = max(0, mc * mx - 1 + gx), x1 = min(sx - 1, mc * mx + mc + gx);
  int y0 = max(0, mc * my - 1 + gy), y1 = min(sy - 1, mc * my + mc + gy);
  int z0 = max(0, mc * mz - 1 + gz), z1 = min(sz - 1, mc * mz + mc + gz);
  int wx = x1 - x0 + 1, wy = y1 - y0 + 1, wz = z1 - z0 + 1;
  int cnt = wx * wy * wz;
  float lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < cnt; i += 256) {
    int x = x0 + i % wx;
    int t = i / wx;
    int y = y0 + t % wy;
    int z = z0 + t / wy;
    float v = load_voxel<T>(vox, blk_x(x) + blk_y(y, bsy) + blk_z(z, bsz));
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o));
    hi = fmaxf(hi, __shfl_xor(hi, o));
  }
  __shared__ float slo[4], shi[4];
  if ((threadIdx.x & 63) == 0) {
    slo[threadIdx.x >> 6] = lo;
    shi[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = fminf(fminf(slo[0], slo[1]), fminf(slo[2], slo[3]));
    float b = fmaxf(fmaxf(shi[0], shi[1]), fmaxf(shi[2], shi[3]));
    ranges[m] = make_float2(a, b);
  }
}

// ------------------------------------------------------------------ majorants
// Largest TF opacity over entries [floor(x_min) - 1, ceil(x_max) + 1] of the range's
// table coordinates x = clamp((v - lo)/(hi - lo), 0, 1) (N - 1), taken in FP32.
__global__ __launch_bounds__(256) void majorant_kernel(const float2* __restrict__ ranges, int count,
                                                       const float4* __restrict__ tf, int ntf, float tf_lo,
                                                       float tf_hi, float* __restrict__ maj) {
  int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= count) return;
  float2 r = ranges[m];
  float span = tf_hi - tf_lo;
  float ua = (r.x - tf_lo) / span;
  float ub = (r.y - tf_lo) / span;
  ua = fminf(fmaxf(ua, 0.f), 1.f);
  ub = fminf(fmaxf(ub, 0.f), 1.f);
  float xa = ua * (float)(ntf - 1);
  float xb = ub * (float)(ntf - 1);
  int e0 = max((int)floorf(xa) - 1, 0);
  int e1 = min((int)ceilf(xb) + 1, ntf - 1);
  float a = 0.f;
  for (int e = e0; e <= e1; ++e) a = fmaxf(a, tf[e].w);
  maj[m] = a;
}

// ------------------------------------------------------------------ ray march
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

template <typename T, bool SKIP>
__device__ __forceinline__ void march_ray(const SceneG& sc, const BrickG& b, const float4* __restrict__ tfb,
                                          const float4* __restrict__ tfs, const double o[3], const double d[3],
                                          float4& out, float& depth, int& nsamp) {
  double lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = b.olo[a] * sc.h;
    hi[a] = b.ohi[a] * sc.h;
  }
  double t_in, t_out;
  if (!clip_box(o, d, lo, hi, t_in, t_out)) {
    out = make_float4(0.f, 0.f, 0.f, 0.f);
    depth = INFINITY;
    nsamp = 0;
    return;
  }
  const double dt = sc.dt;
  const int s0 = (int)floor(t_in / dt);
  const int s1 = (int)ceil(t_out / dt) - 1;
  double ov[3], dv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ov[a] = o[a] * sc.inv_h - 0.5;
    dv[a] = d[a] * sc.inv_h;
  }
  const T* vox = (const T*)b.data;
  const double nx1 = sc.dims[0] - 1, ny1 = sc.dims[1] - 1, nz1 = sc.dims[2] - 1;
  const float Ddt = sc.density * sc.dt_f;
  float cr = 0.f, cg = 0.f, cb = 0.f, tr = 1.f;
  double tau_acc = 0.0;
  int n = 0;
  for (int s = s0; s <= s1; ++s) {
    const double tlo = (double)s * dt;
    const double thi = tlo + dt;
    float Dl = Ddt;
    if (tlo < t_in || thi > t_out) {
      double l = fmin(thi, t_out) - fmax(tlo, t_in);
      if (!(l > 0.0)) continue;
      Dl = sc.density * (float)l;
    }
    ++n;
    const double tm = tlo + 0.5 * dt;
    const double gx = fma(tm, dv[0], ov[0]);
    const double gy = fma(tm, dv[1], ov[1]);
    const double gz = fma(tm, dv[2], ov[2]);
    if (SKIP) {
      int mx = ((int)floor(gx + 0.5) - b.olo[0]) >> b.mc_shift;
      int my = ((int)floor(gy + 0.5) - b.olo[1]) >> b.mc_shift;
      int mz = ((int)floor(gz + 0.5) - b.olo[2]) >> b.mc_shift;
      mx = min(max(mx, 0), b.mdim[0] - 1);
      my = min(max(my, 0), b.mdim[1] - 1);
      mz = min(max(mz, 0), b.mdim[2] - 1);
      if (b.majorant[(mz * b.mdim[1] + my) * b.mdim[0] + mx] == 0.f) continue;
    }
    const double cx = fmin(fmax(gx, 0.0), nx1);
    const double cy = fmin(fmax(gy, 0.0), ny1);
    const double cz = fmin(fmax(gz, 0.0), nz1);
    const int ix = min((int)floor(cx), sc.dims[0] - 2);
    const int iy = min((int)floor(cy), sc.dims[1] - 2);
    const int iz = min((int)floor(cz), sc.dims[2] - 2);
    const float fx = (float)(cx - ix), fy = (float)(cy - iy), fz = (float)(cz - iz);
    // commit guarantees these lie in [0, sdim - 2]; the clamp only guards memory
    const int lx = min(max(ix - b.slo[0], 0), b.sdim[0] - 2);
    const int ly = min(max(iy - b.slo[1], 0), b.sdim[1] - 2);
    const int lz = min(max(iz - b.slo[2], 0), b.sdim[2] - 2);
    const uint32_t x0 = blk_x(lx), x1 = blk_x(lx + 1);
    const uint32_t y0 = blk_y(ly, b.bsy), y1 = blk_y(ly + 1, b.bsy);
    const uint32_t z0 = blk_z(lz, b.bsz), z1 = blk_z(lz + 1, b.bsz);
    const float v000 = load_voxel<T>(vox, x0 + y0 + z0), v001 = load_voxel<T>(vox, x1 + y0 + z0);
    const float v010 = load_voxel<T>(vox, x0 + y1 + z0), v011 = load_voxel<T>(vox, x1 + y1 + z0);
    const float v100 = load_voxel<T>(vox, x0 + y0 + z1), v101 = load_voxel<T>(vox, x1 + y0 + z1);
    const float v110 = load_voxel<T>(vox, x0 + y1 + z1), v111 = load_voxel<T>(vox, x1 + y1 + z1);
    const float c00 = fmaf(fx, v001 - v000, v000), c01 = fmaf(fx, v011 - v010, v010);
    const float c10 = fmaf(fx, v101 - v100, v100), c11 = fmaf(fx, v111 - v110, v110);
    const float c0 = fmaf(fy, c01 - c00, c00), c1 = fmaf(fy, c11 - c10, c10);
    const float v = fmaf(fz, c1 - c0, c0);
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
      if (1.f - tr >= sc.ert) break;
    }
  }
  out = make_float4(cr, cg, cb, 1.f - tr);
  depth = (float)t_in;
  nsamp = n;
}

// Plain per-brick launch: one thread per pixel, 16x16 tiles as four 8x8 waves,
// tiles assigned so that each XCD (round-robin workgroup dispatch) walks one
// contiguous band of the screen and keeps its part of the brick in its own L2.
template <typename T, bool SKIP>
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
  float4 c;
  float z;
  int n;
  march_ray<T, SKIP>(sc, b, tfb, tfs, cam.eye, d, c, z, n);
  const size_t p = (size_t)py * cam.W + px;
  out_rgba[p] = c;
  out_depth[p] = z;
  if (out_count) out_count[p] = n;
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_relayout(const void* src, void* dst, int elem_bytes, int sx, int sy, int sz, int bx, int by,
                           int bz, hipStream_t st) {
  uint64_t total = (uint64_t)bx * by * bz * kBlockVoxels;
  dim3 grid((unsigned)((total + 255) / 256));
  if (elem_bytes == 4)
    hipLaunchKernelGGL(relayout_kernel<uint32_t>, grid, dim3(256), 0, st, (const uint32_t*)src, (uint32_t*)dst, sx,
                       sy, sz, bx, by, total);
  else
    hipLaunchKernelGGL(relayout_kernel<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)src, (uint16_t*)dst, sx,
                       sy, sz, bx, by, total);
  return hipGetLastError();
}

hipError_t launch_macrocells(const BrickG& b, bool f16, int mc, float2* ranges, hipStream_t st) {
  int count = b.mdim[0] * b.mdim[1] * b.mdim[2];
  int gx = b.olo[0] - b.slo[0], gy = b.olo[1] - b.slo[1], gz = b.olo[2] - b.slo[2];
  if (f16)
    hipLaunchKernelGGL(macrocell_kernel<__half>, dim3(count), dim3(256), 0, st, (const __half*)b.data, b.sdim[0],
                       b.sdim[1], b.sdim[2], b.bsy, b.bsz, gx, gy, gz, mc, b.mdim[0], b.mdim[1], b.mdim[2], ranges);
  else
    hipLaunchKernelGGL(macrocell_kernel<float>, dim3(count), dim3(256), 0, st, (const float*)b.data, b.sdim[0],
                       b.sdim[1], b.sdim[2], b.bsy, b.bsz, gx, gy, gz, mc, b.mdim[0], b.mdim[1], b.mdim[2], ranges);
  return hipGetLastError();
}

hipError_t launch_majorants(const float2* ranges, int count, const float4* tf, int ntf, float lo, float hi,
                            float* maj, hipStream_t st) {
  hipLaunchKernelGGL(majorant_kernel, dim3((count + 255) / 256), dim3(256), 0, st, ranges, count, tf, ntf, lo, hi,
                     maj);
  return hipGetLastError();
}

hipError_t launch_march(const SceneG& sc, const BrickG& b, const CamG& cam, const float4* tf, bool f16, bool skip,
                        float4* rgba, float* depth, int* count, hipStream_t st) {
  int tx = (cam.W + 15) / 16, ty = (cam.H + 15) / 16;
  int n_tiles = tx * ty;
  int nb = ((n_tiles + 7) / 8) * 8;
  dim3 grid(nb), block(256);
  size_t lds = 2 * sizeof(float4) * (size_t)sc.ntf;
  if (f16) {
    if (skip)
      hipLaunchKernelGGL((march_kernel<__half, true>), grid, block, lds, st, sc, b, cam, tf, rgba, depth, count, tx,
                         n_tiles);
    else
      hipLaunchKernelGGL((march_kernel<__half, false>), grid, block, lds, st, sc, b, cam, tf, rgba, depth, count, tx,
                         n_tiles);
  } else {
    if (skip)
      hipLaunchKernelGGL((march_kernel<float, true>), grid, block, lds, st, sc, b, cam, tf, rgba, depth, count, tx,
                         n_tiles);
    else
      hipLaunchKernelGGL((march_kernel<float, false>), grid, block, lds, st, sc, b, cam, tf, rgba, depth, count, tx,
                         n_tiles);
  }
  return hipGetLastError();
}

}  // namespace dpr
