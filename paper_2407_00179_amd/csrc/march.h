// Resumable per-ray emission-absorption march through one brick.
//
// The plain per-brick kernel runs a ray to completion in one call; the
// persistent batched kernel advances rays a few segments at a time so a wave can
// refill lanes whose rays have finished.  Both use exactly this code, so both
// produce the same bits for the same ray.
#pragma once

#include "device_common.h"

namespace dpr {

struct RayState {
  double ov[3], dv[3];   // origin and direction in global voxel-centre units
  double t_in, t_out;    // clipped parametric range (world units)
  double tau;            // optical depth accumulated so far
  int s, s1;             // next lattice segment, last lattice segment
  int n;                 // logical samples processed
  float T, cr, cg, cb;   // transmittance and premultiplied colour
};

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
  r.s = (int)floor(r.t_in / sc.dt);
  r.s1 = (int)ceil(r.t_out / sc.dt) - 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.ov[a] = o[a] * sc.inv_h - 0.5;
    r.dv[a] = d[a] * sc.inv_h;
  }
  r.tau = 0.0;
  r.n = 0;
  r.T = 1.f;
  r.cr = r.cg = r.cb = 0.f;
  return true;
}

// Advance by at most `budget` lattice segments.  Returns true once the ray is
// finished: past its last segment, or terminated early (1 - T >= ert, tested
// after every segment that changed T).
template <typename T, bool SKIP>
__device__ __forceinline__ bool ray_advance(const SceneG& sc, const BrickG& b, const float4* __restrict__ tfb,
                                            const float4* __restrict__ tfs, RayState& r, int budget) {
  const double dt = sc.dt;
  const T* vox = (const T*)b.data;
  const double nx1 = sc.dims[0] - 1, ny1 = sc.dims[1] - 1, nz1 = sc.dims[2] - 1;
  const float Ddt = sc.density * sc.dt_f;
  int s = r.s;
  const int s1 = r.s1;
  const int s_end = (s1 - s < budget) ? s1 : s + budget - 1;
  float tr = r.T, cr = r.cr, cg = r.cg, cb = r.cb;
  double tau_acc = r.tau;
  int n = r.n;
  bool done = false;
  for (; s <= s_end; ++s) {
    const double tlo = (double)s * dt;
    const double thi = tlo + dt;
    float Dl = Ddt;
    if (tlo < r.t_in || thi > r.t_out) {
      double l = fmin(thi, r.t_out) - fmax(tlo, r.t_in);
      if (!(l > 0.0)) continue;
      Dl = sc.density * (float)l;
    }
    ++n;
    const double tm = tlo + 0.5 * dt;
    const double gx = fma(tm, r.dv[0], r.ov[0]);
    const double gy = fma(tm, r.dv[1], r.ov[1]);
    const double gz = fma(tm, r.dv[2], r.ov[2]);
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
      if (1.f - tr >= sc.ert) {
        done = true;
        ++s;
        break;
      }
    }
  }
  r.s = s;
  r.T = tr;
  r.cr = cr;
  r.cg = cg;
  r.cb = cb;
  r.tau = tau_acc;
  r.n = n;
  return done || s > s1;
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
