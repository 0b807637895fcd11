// Differentiable emission-absorption render of one whole FP32 volume (ERT off, no
// skipping) and its hand-written adjoint.
//
// Forward: the same quadrature as the brick renderer (32.32 fixed-point sample
// points, trilinear, TF lerp, tau = D A l, T = exp(-sum tau)), storing per ray the
// total optical depth and a checkpoint of the optical depth before every 64th
// segment.
// Backward: per ray, segments are visited in reverse.  Transmittance is never
// stored per sample: the optical depth before a segment is the one after it minus
// its own tau (recomputed from the volume), and it is reset to the stored value at
// every checkpoint.  With g_C = dL/dC, g_a = dL/dalpha and C_{>s} the colour of the
// segments behind s (accumulated on the way back):
//   dL/dc_s   = T_s (1 - e^{-tau_s}) g_C
//   dL/dtau_s = g_C . (T_{s+1} c_s - C_{>s}) + g_a T_S,   dL/dA_s = dL/dtau_s D l_s
// The TF gradient goes to the two lerp entries (weights 1-w, w) through an
// LDS-private copy flushed once per workgroup; the volume gradient goes to the 8
// trilinear corners with global atomics, pre-summed in registers while consecutive
// samples share the same cell, and carried over for the corners that the next
// cell shares with it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "march.h"
#include "runtime.hpp"

namespace dpr {

constexpr int kCkpt = 64;  // segments per checkpoint

struct TrainG {
  int dims[3];
  double h, inv_h, dt;
  float dt_f, density, tf_lo, tf_scale;
  int ntf;
  int W, H, n_cams;
  int ws_stride;  // doubles per ray: total optical depth + checkpoints
};

struct TrainRay {
  int64_t p[3], dp[3];
  double t_in, t_out;
  int s0, s1;
  float dl_first, dl_last;
};

__device__ __forceinline__ bool train_begin(const TrainG& g, const double o[3], const double d[3], TrainRay& r) {
  const double lo[3] = {0.0, 0.0, 0.0};
  const double hi[3] = {g.dims[0] * g.h, g.dims[1] * g.h, g.dims[2] * g.h};
  if (!clip_box(o, d, lo, hi, r.t_in, r.t_out)) return false;
  const double dt = g.dt;
  int s0 = (int)floor(r.t_in / dt);
  int s1 = (int)ceil(r.t_out / dt) - 1;
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
  r.s0 = s0;
  r.s1 = s1;
  r.dl_first = g.density * (float)lf;
  r.dl_last = g.density * (float)ll;
  const double tm = (s0 + 0.5) * dt;
  for (int a = 0; a < 3; ++a) {
    const double dv = d[a] * g.inv_h;
    r.p[a] = __double2ll_rn(fma(tm, dv, o[a] * g.inv_h - 0.5) * kFix);
    r.dp[a] = __double2ll_rn(dt * dv * kFix);
  }
  return true;
}

// Trilinear stencil of a fixed-point point in the global volume (clamp-to-edge).
struct Stencil {
  int i, j, k;  // base corner
  float fx, fy, fz;
};

__device__ __forceinline__ void stencil_axis(int64_t p, int n, int& i0, float& f) {
  const int hi = (int)(p >> 32);
  float fr = (float)(uint32_t)(p & 0xffffffffll) * (1.0f / 4294967296.0f);
  f = (hi < 0) ? 0.f : ((hi > n - 2) ? 1.f : fr);
  i0 = min(max(hi, 0), n - 2);
}

__device__ __forceinline__ float sample_linear(const float* __restrict__ vol, const TrainG& g, const int64_t p[3],
                                               Stencil& st) {
  stencil_axis(p[0], g.dims[0], st.i, st.fx);
  stencil_axis(p[1], g.dims[1], st.j, st.fy);
  stencil_axis(p[2], g.dims[2], st.k, st.fz);
  const size_t sx = 1, sy = (size_t)g.dims[0], sz = (size_t)g.dims[0] * g.dims[1];
  const size_t b = st.k * sz + st.j * sy + st.i;
  const float v000 = vol[b], v001 = vol[b + sx], v010 = vol[b + sy], v011 = vol[b + sy + sx];
  const float v100 = vol[b + sz], v101 = vol[b + sz + sx], v110 = vol[b + sz + sy], v111 = vol[b + sz + sy + sx];
  const float c00 = fmaf(st.fx, v001 - v000, v000), c01 = fmaf(st.fx, v011 - v010, v010);
  const float c10 = fmaf(st.fx, v101 - v100, v100), c11 = fmaf(st.fx, v111 - v110, v110);
  const float c0 = fmaf(st.fy, c01 - c00, c00), c1 = fmaf(st.fy, c11 - c10, c10);
  return fmaf(st.fz, c1 - c0, c0);
}

__global__ __launch_bounds__(256) void train_forward_kernel(TrainG g, const CamG* __restrict__ cams,
                                                            const float* __restrict__ vol,
                                                            const float4* __restrict__ tf, float4* __restrict__ out,
                                                            float* __restrict__ out_depth, double* __restrict__ ws,
                                                            int tiles_x, int tiles_per_cam) {
  extern __shared__ float4 lds[];
  float4* tfb = lds;
  float4* tfs = lds + g.ntf;
  stage_tf(tf, g.ntf, tfb, tfs, threadIdx.x, 256);
  __syncthreads();
  const int cam_id = blockIdx.x / tiles_per_cam;
  const int tile = blockIdx.x % tiles_per_cam;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = (tile % tiles_x) * 16 + (wave & 1) * 8 + (lane & 7);
  const int py = (tile / tiles_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
  if (px >= g.W || py >= g.H) return;
  const CamG& cam = cams[cam_id];
  const size_t ray = ((size_t)cam_id * g.H + py) * g.W + px;
  double* w = ws + ray * g.ws_stride;
  double d[3];
  camera_ray(cam, px, py, d);
  TrainRay r;
  if (!train_begin(g, cam.eye, d, r)) {
    out[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
    out_depth[ray] = INFINITY;
    w[0] = 0.0;
    return;
  }
  int64_t p[3] = {r.p[0], r.p[1], r.p[2]};
  const float Ddt = g.density * g.dt_f;
  double tau_acc = 0.0;
  float tr = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
  for (int s = r.s0; s <= r.s1; ++s) {
    const int k = s - r.s0;
    if ((k & (kCkpt - 1)) == 0) w[1 + k / kCkpt] = tau_acc;
    Stencil st;
    const float v = sample_linear(vol, g, p, st);
    p[0] += r.dp[0];
    p[1] += r.dp[1];
    p[2] += r.dp[2];
    float x = (v - g.tf_lo) * g.tf_scale;
    x = fminf(fmaxf(x, 0.f), (float)(g.ntf - 1));
    const int j = min((int)x, g.ntf - 2);
    const float wl = x - (float)j;
    const float4 tb = tfb[j], ts = tfs[j];
    const float A = fmaf(wl, ts.w, tb.w);
    const float Dl = (s == r.s0) ? r.dl_first : ((s == r.s1) ? r.dl_last : Ddt);
    const float tau = Dl * A;
    if (tau > 0.f) {
      tau_acc += (double)tau;
      const float tn = __expf(-(float)tau_acc);
      const float wgt = tr - tn;
      cr = fmaf(wgt, fmaf(wl, ts.x, tb.x), cr);
      cg = fmaf(wgt, fmaf(wl, ts.y, tb.y), cg);
      cb = fmaf(wgt, fmaf(wl, ts.z, tb.z), cb);
      tr = tn;
    }
  }
  w[0] = tau_acc;
  out[ray] = make_float4(cr, cg, cb, 1.f - tr);
  out_depth[ray] = (float)r.t_in;
}

__device__ __forceinline__ void flush_corners(float* __restrict__ gvol, const TrainG& g, const Stencil& st,
                                              const float acc[8]) {
  const size_t sx = 1, sy = (size_t)g.dims[0], sz = (size_t)g.dims[0] * g.dims[1];
  const size_t b = st.k * sz + st.j * sy + st.i;
  const size_t off[8] = {0, sx, sy, sy + sx, sz, sz + sx, sz + sy, sz + sy + sx};
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (acc[c] != 0.f) atomicAdd(gvol + b + off[c], acc[c]);
}

// The ray's trilinear cell moved from `cur` by (dx, dy, dz), each in {-1, 0, 1}
// (a step of at most one voxel).  Corners the old and new cells share keep their
// sums, moved to their slots in the new cell (slot x + 2 y + 4 z); the others are
// added to the volume gradient.  A move along one axis thus flushes 4 corners,
// not 8.
__device__ __forceinline__ void carry_corners(float* __restrict__ gvol, const TrainG& g, const Stencil& cur,
                                              float acc[8], int dx, int dy, int dz) {
  const size_t sx = 1, sy = (size_t)g.dims[0], sz = (size_t)g.dims[0] * g.dims[1];
  const size_t b = cur.k * sz + cur.j * sy + cur.i;
  const size_t off[8] = {0, sx, sy, sy + sx, sz, sz + sx, sz + sy, sz + sy + sx};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const bool keep = (unsigned)((c & 1) - dx) <= 1u && (unsigned)(((c >> 1) & 1) - dy) <= 1u &&
                      (unsigned)((c >> 2) - dz) <= 1u;
    if (!keep && acc[c] != 0.f) atomicAdd(gvol + b + off[c], acc[c]);
  }
  // new slot (x, y, z) <- old slot (x + dx, y + dy, z + dz), zero outside the old cell;
  // one axis at a time (slot pairs 1, 2 and 4 apart)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int d = a == 0 ? dx : (a == 1 ? dy : dz);
    const int st = 1 << a;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c & st) continue;
      const float o0 = acc[c], o1 = acc[c + st];
      acc[c] = d == 0 ? o0 : (d > 0 ? o1 : 0.f);
      acc[c + st] = d == 0 ? o1 : (d < 0 ? o0 : 0.f);
    }
  }
}

// TF-gradient replicas in LDS: lanes add into replica (lane & 7); replicas are
// padded by one float so the same entry of different replicas falls in different
// banks.  This cuts same-address atomic conflicts (many lanes hit the same few
// entries, e.g. the transparent floor) by 8x.
constexpr int kTfRep = 8;

__device__ __forceinline__ void lds_add(float* p, float v) {
  if (v != 0.f) atomicAdd(p, v);
}

__global__ __launch_bounds__(256) void train_backward_kernel(TrainG g, const CamG* __restrict__ cams,
                                                             const float* __restrict__ vol,
                                                             const float4* __restrict__ tf,
                                                             const float4* __restrict__ grad_out,
                                                             const double* __restrict__ ws,
                                                             float* __restrict__ gvol, double* __restrict__ gtf,
                                                             int tiles_x, int tiles_per_cam) {
  extern __shared__ float4 lds[];
  float4* tfb = lds;
  float4* tfs = lds + g.ntf;
  float* gt = (float*)(lds + 2 * g.ntf);  // kTfRep replicas of 4 * ntf floats, stride 4 * ntf + 1
  const int rstride = 4 * g.ntf + 1;
  stage_tf(tf, g.ntf, tfb, tfs, threadIdx.x, 256);
  for (int i = threadIdx.x; i < kTfRep * rstride; i += 256) gt[i] = 0.f;
  __syncthreads();
  const int cam_id = blockIdx.x / tiles_per_cam;
  const int tile = blockIdx.x % tiles_per_cam;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = (tile % tiles_x) * 16 + (wave & 1) * 8 + (lane & 7);
  const int py = (tile / tiles_x) * 16 + (wave >> 1) * 8 + (lane >> 3);
  const float slope_scale = g.tf_scale;
  float* my_gt = gt + (lane & (kTfRep - 1)) * rstride;
  if (px < g.W && py < g.H) {
    const CamG& cam = cams[cam_id];
    const size_t ray = ((size_t)cam_id * g.H + py) * g.W + px;
    const double* w = ws + ray * g.ws_stride;
    double d[3];
    camera_ray(cam, px, py, d);
    TrainRay r;
    const float4 go = grad_out[ray];
    if (train_begin(g, cam.eye, d, r) && r.s1 >= r.s0 &&
        (go.x != 0.f || go.y != 0.f || go.z != 0.f || go.w != 0.f)) {
      const double tau_total = w[0];
      const float T_S = __expf(-(float)tau_total);
      const float Ddt = g.density * g.dt_f;
      float sr = 0.f, sg = 0.f, sb = 0.f;  // C_{>s}
      double tau_after = tau_total;
      float T_next = T_S;  // transmittance after the current segment
      Stencil cur;
      cur.i = -1;
      float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      // sample point of the last segment; stepping back by dp gives exactly the
      // forward's points (fixed-point integers)
      int64_t p[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) p[a] = r.p[a] + (int64_t)(r.s1 - r.s0) * r.dp[a];
      for (int s = r.s1; s >= r.s0; --s) {
        const int k = s - r.s0;
        // top of a chunk: optical depth after this segment from the forward's record
        if (((k + 1) & (kCkpt - 1)) == 0 && s != r.s1) {
          tau_after = w[1 + (k + 1) / kCkpt];
          T_next = __expf(-(float)tau_after);
        }
        Stencil st;
        const float v = sample_linear(vol, g, p, st);
        const float xr = (v - g.tf_lo) * g.tf_scale;
        const float x = fminf(fmaxf(xr, 0.f), (float)(g.ntf - 1));
        const int j = min((int)x, g.ntf - 2);
        const float wl = x - (float)j;
        const float4 tb = tfb[j], ts = tfs[j];
        const float A = fmaf(wl, ts.w, tb.w);
        const float cR = fmaf(wl, ts.x, tb.x), cG = fmaf(wl, ts.y, tb.y), cB = fmaf(wl, ts.z, tb.z);
        const float Dl = (s == r.s0) ? r.dl_first : ((s == r.s1) ? r.dl_last : Ddt);
        const float tau = Dl * A;
        float T_s = T_next, wgt = 0.f;
        double tau_before = tau_after;
        if (tau > 0.f) {
          tau_before = tau_after - (double)tau;
          T_s = __expf(-(float)tau_before);
          // per-sample weight T_s (1 - e^-tau) with expm1: exact even for tau ~ 1e-5,
          // where the difference T_s - T_{s+1} would lose most of its digits
          wgt = -T_s * expm1f(-tau);
        }
        // dL/dc_s and dL/dA_s
        const float gcR = wgt * go.x, gcG = wgt * go.y, gcB = wgt * go.z;
        const float gtau = go.x * (T_next * cR - sr) + go.y * (T_next * cG - sg) + go.z * (T_next * cB - sb) +
                           go.w * T_S;
        const float gA = gtau * Dl;
        sr = fmaf(wgt, cR, sr);
        sg = fmaf(wgt, cG, sg);
        sb = fmaf(wgt, cB, sb);
        tau_after = tau_before;
        T_next = T_s;
        // TF entries j, j+1 (colour terms vanish where the sample is transparent)
        float* e0 = my_gt + 4 * j;
        const float w0 = 1.f - wl;
        if (wgt != 0.f) {
          lds_add(e0 + 0, w0 * gcR);
          lds_add(e0 + 1, w0 * gcG);
          lds_add(e0 + 2, w0 * gcB);
          lds_add(e0 + 4, wl * gcR);
          lds_add(e0 + 5, wl * gcG);
          lds_add(e0 + 6, wl * gcB);
        }
        lds_add(e0 + 3, w0 * gA);
        lds_add(e0 + 7, wl * gA);
        // sample value: zero outside the TF range (clamped u)
        const bool inside = xr >= 0.f && xr <= (float)(g.ntf - 1);
        const float gv = inside ? (gA * ts.w + gcR * ts.x + gcG * ts.y + gcB * ts.z) * slope_scale : 0.f;
        if (st.i != cur.i || st.j != cur.j || st.k != cur.k) {
          const int dx = st.i - cur.i, dy = st.j - cur.j, dz = st.k - cur.k;
          if (cur.i >= 0 && abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) {
            carry_corners(gvol, g, cur, acc, dx, dy, dz);
          } else {
            if (cur.i >= 0) flush_corners(gvol, g, cur, acc);
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] = 0.f;
          }
          cur = st;
        }
        const float ux = st.fx, uy = st.fy, uz = st.fz;
        const float lx = 1.f - ux, ly = 1.f - uy, lz = 1.f - uz;
        acc[0] = fmaf(gv, lz * ly * lx, acc[0]);
        acc[1] = fmaf(gv, lz * ly * ux, acc[1]);
        acc[2] = fmaf(gv, lz * uy * lx, acc[2]);
        acc[3] = fmaf(gv, lz * uy * ux, acc[3]);
        acc[4] = fmaf(gv, uz * ly * lx, acc[4]);
        acc[5] = fmaf(gv, uz * ly * ux, acc[5]);
        acc[6] = fmaf(gv, uz * uy * lx, acc[6]);
        acc[7] = fmaf(gv, uz * uy * ux, acc[7]);
#pragma unroll
        for (int a = 0; a < 3; ++a) p[a] -= r.dp[a];
      }
      if (cur.i >= 0) flush_corners(gvol, g, cur, acc);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * g.ntf; i += 256) {
    float v = 0.f;
#pragma unroll
    for (int rep = 0; rep < kTfRep; ++rep) v += gt[rep * rstride + i];
    // the workgroups' partial sums meet in FP64, so an entry's error is that of
    // one workgroup's FP32 sum, not of thousands of rounded additions
    if (v != 0.f) atomicAdd(gtf + i, (double)v);
  }
}

__global__ void fill_f64_kernel(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// grad_tf += the FP64 sums (rounded once to FP32)
__global__ void add_f64_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += (float)src[i];
}

static int max_segments(const int64_t dims[3], float step) {
  const double m = (double)std::max(dims[0], std::max(dims[1], dims[2]));
  const double diag = std::sqrt((double)dims[0] * dims[0] + (double)dims[1] * dims[1] + (double)dims[2] * dims[2]) / m;
  return (int)std::ceil(diag / (step / m)) + 3;
}

static dpr_status check_train(const int64_t dims[3], const dpr_camera* cams, int n, const dpr_render_params* prm,
                              int n_tf, float lo, float hi, float density) {
  if (!dims || !cams || !prm) return fail(DPR_ERR_INVALID_ARGUMENT, "training call: NULL argument");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 2 || dims[a] > (1 << 16)) return fail(DPR_ERR_INVALID_ARGUMENT, "training call: dims[%d]", a);
  if (n < 1) return fail(DPR_ERR_INVALID_ARGUMENT, "training call: n = %d", n);
  for (int c = 0; c < n; ++c) {
    dpr_status s = check_camera(&cams[c]);
    if (s != DPR_OK) return s;
    if (cams[c].width != cams[0].width || cams[c].height != cams[0].height)
      return fail(DPR_ERR_INVALID_ARGUMENT, "training call: all cameras must share one image size");
  }
  if (!(prm->step_voxels > 0.f && prm->step_voxels <= 1.f))
    return fail(DPR_ERR_INVALID_ARGUMENT, "training call: step_voxels %g", prm->step_voxels);
  if (n_tf < 2 || n_tf > kMaxTF) return fail(DPR_ERR_INVALID_ARGUMENT, "training call: n_tf %d", n_tf);
  if (!(hi > lo)) return fail(DPR_ERR_INVALID_ARGUMENT, "training call: value range");
  if (!(density >= 0.f)) return fail(DPR_ERR_INVALID_ARGUMENT, "training call: density");
  return DPR_OK;
}

static TrainG make_train(const int64_t dims[3], const dpr_camera* cams, int n, const dpr_render_params* prm, int n_tf,
                         float lo, float hi, float density) {
  TrainG g{};
  int64_t m = std::max(dims[0], std::max(dims[1], dims[2]));
  for (int a = 0; a < 3; ++a) g.dims[a] = (int)dims[a];
  g.h = 1.0 / (double)m;
  g.inv_h = (double)m;
  g.dt = (double)prm->step_voxels * g.h;
  g.dt_f = (float)g.dt;
  g.density = density;
  g.tf_lo = lo;
  g.tf_scale = (float)(n_tf - 1) / (hi - lo);
  g.ntf = n_tf;
  g.W = cams[0].width;
  g.H = cams[0].height;
  g.n_cams = n;
  g.ws_stride = 1 + (max_segments(dims, prm->step_voxels) + kCkpt - 1) / kCkpt;
  return g;
}

// Camera tables of the training calls, cached per device by content.
struct CamCacheEntry {
  dpr_device dev;
  int hip_device;
  std::vector<dpr_camera> cams;
  CamG* table;
};

static dpr_status cam_table(dpr_device dev, const dpr_camera* cams, int n, CamG** out) {
  static thread_local std::vector<CamCacheEntry> cache;
  for (auto& e : cache)
    if (e.dev == dev && e.hip_device == dev->dev && (int)e.cams.size() == n &&
        memcmp(e.cams.data(), cams, n * sizeof(dpr_camera)) == 0) {
      *out = e.table;
      return DPR_OK;
    }
  std::vector<CamG> h(n);
  for (int c = 0; c < n; ++c) h[c] = make_cam(cams[c]);
  CamG* d = nullptr;
  dpr_status s = dev_alloc((void**)&d, n * sizeof(CamG), "training cameras");
  if (s != DPR_OK) return s;
  DPR_HIP(hipMemcpyAsync(d, h.data(), n * sizeof(CamG), hipMemcpyHostToDevice, dev->stream));
  DPR_HIP(hipStreamSynchronize(dev->stream));
  if (cache.size() >= 16) {
    DPR_HIP(hipStreamSynchronize(dev->stream));
    dev_free(cache.front().table);
    cache.erase(cache.begin());
  }
  cache.push_back({dev, dev->dev, std::vector<dpr_camera>(cams, cams + n), d});
  *out = d;
  return DPR_OK;
}

}  // namespace dpr

using namespace dpr;

extern "C" {

dpr_status dpr_train_workspace_size(const int64_t dims[3], const dpr_camera* cams, int32_t n, float step,
                                    size_t* bytes) {
  if (!dims || !cams || !bytes) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_train_workspace_size: NULL argument");
  dpr_render_params p{step, 2.f, 16, 0u};
  dpr_status s = check_train(dims, cams, n, &p, 2, 0.f, 1.f, 0.f);
  if (s != DPR_OK) return s;
  TrainG g = make_train(dims, cams, n, &p, 2, 0.f, 1.f, 0.f);
  *bytes = (size_t)n * g.W * g.H * g.ws_stride * sizeof(double);
  return DPR_OK;
}

dpr_status dpr_render_train_forward(dpr_device dev, const float* volume, const int64_t dims[3], const float* tf,
                                    int32_t n_tf, float lo, float hi, float density, const dpr_render_params* prm,
                                    const dpr_camera* cams, int32_t n, float* out_rgba, float* out_depth,
                                    void* ws, size_t ws_bytes) {
  if (!dev || !volume || !tf || !out_rgba || !out_depth || !ws)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_train_forward: NULL argument");
  dpr_status s = check_train(dims, cams, n, prm, n_tf, lo, hi, density);
  if (s != DPR_OK) return s;
  TrainG g = make_train(dims, cams, n, prm, n_tf, lo, hi, density);
  size_t need = (size_t)n * g.W * g.H * g.ws_stride * sizeof(double);
  if (ws_bytes < need)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_train_forward: workspace %zu < %zu bytes", ws_bytes, need);
  CamG* dc = nullptr;
  if ((s = cam_table(dev, cams, n, &dc)) != DPR_OK) return s;
  const int tx = (g.W + 15) / 16, ty = (g.H + 15) / 16;
  dim3 grid((unsigned)(tx * ty * n));
  size_t lds = 2 * sizeof(float4) * (size_t)n_tf;
  hipLaunchKernelGGL(train_forward_kernel, grid, dim3(256), lds, dev->stream, g, dc, volume, (const float4*)tf,
                     (float4*)out_rgba, out_depth, (double*)ws, tx, tx * ty);
  DPR_HIP(hipGetLastError());
  return DPR_OK;
}

dpr_status dpr_render_backward(dpr_device dev, const float* volume, const int64_t dims[3], const float* tf,
                               int32_t n_tf, float lo, float hi, float density, const dpr_render_params* prm,
                               const dpr_camera* cams, int32_t n, const float* grad_rgba, const void* ws,
                               size_t ws_bytes, float* grad_volume, float* grad_tf) {
  if (!dev || !volume || !tf || !grad_rgba || !ws || !grad_volume || !grad_tf)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_backward: NULL argument");
  dpr_status s = check_train(dims, cams, n, prm, n_tf, lo, hi, density);
  if (s != DPR_OK) return s;
  TrainG g = make_train(dims, cams, n, prm, n_tf, lo, hi, density);
  size_t need = (size_t)n * g.W * g.H * g.ws_stride * sizeof(double);
  if (ws_bytes < need)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_backward: workspace %zu < %zu bytes", ws_bytes, need);
  CamG* dc = nullptr;
  if ((s = cam_table(dev, cams, n, &dc)) != DPR_OK) return s;
  const int tx = (g.W + 15) / 16, ty = (g.H + 15) / 16;
  dim3 grid((unsigned)(tx * ty * n));
  if (!dev->tf_grad64 && (s = dev_alloc((void**)&dev->tf_grad64, 4 * kMaxTF * sizeof(double),
                                           "transfer-function gradient sums")) != DPR_OK)
    return s;
  const int nt = 4 * n_tf;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((nt + 255) / 256), dim3(256), 0, dev->stream, dev->tf_grad64, nt);
  size_t lds = 2 * sizeof(float4) * (size_t)n_tf + sizeof(float) * (size_t)kTfRep * (4 * n_tf + 1);
  hipLaunchKernelGGL(train_backward_kernel, grid, dim3(256), lds, dev->stream, g, dc, volume, (const float4*)tf,
                     (const float4*)grad_rgba, (const double*)ws, grad_volume, dev->tf_grad64, tx, tx * ty);
  hipLaunchKernelGGL(add_f64_to_f32_kernel, dim3((nt + 255) / 256), dim3(256), 0, dev->stream, dev->tf_grad64,
                     grad_tf, nt);
  DPR_HIP(hipGetLastError());
  return DPR_OK;
}

}  // extern "C"
