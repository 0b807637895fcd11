// Batched rendering of many cameras over uneven bricks.
//
// One persistent launch walks a queue of (camera, brick, screen tile) items.
// Each wave pops an item with one atomic, takes its rays as a pool, and marches
// them a few segments at a time; lanes whose ray has finished (left the brick or
// terminated early) write their fragment and are refilled from the pool with
// ballot/popcount compaction, so a wave is not held back by its longest ray.  A
// wave keeps one (camera, brick) at a time so brick and camera descriptors stay
// wave-uniform.  A tile compositor then merges, per camera tile, the fragments of
// every item covering it.  Reset + march + composite are captured once into a
// HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "composite.h"
#include "march.h"
#include "runtime.hpp"

namespace dpr {

struct BatchItem {
  int cam, brick, tx, ty;
};

struct BatchG {
  const CamG* cams;
  const BrickG* bricks;
  const BatchItem* items;
  int n_items;
  int tile_w, tile_h;
  float4* frag_rgba;
  float* frag_depth;
  int* head;
  int* item_count;  // coverage counters (DPR_FLAG_QUEUE_COVERAGE), else null
  int* slot_count;
};

// Segments between refill checks.  A return to the refill point costs a ballot,
// the pool bookkeeping and a fresh exact macrocell-run computation, so checks are
// kept rare; a lane that finishes early waits at most this many segments.
constexpr int kChunk = 128;
constexpr int kRefillLanes = 32;

__global__ void reset_head_kernel(int* head) { *head = 0; }
__global__ void zero_counts_kernel(int* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

template <typename T, bool SKIP, bool WIDE, bool ISO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void batch_march_kernel(SceneG sc, BatchG bg, const float4* __restrict__ tf) {
  extern __shared__ float4 tf_lds[];
  float4* tfb = tf_lds;
  float4* tfs = tf_lds + sc.ntf;
  stage_tf(tf, sc.ntf, tfb, tfs, threadIdx.x, 256);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int tp = bg.tile_w * bg.tile_h;

  int cur_cam = -1, cur_brick = -1;
  int pool_item = -1, pool_next = 0, pool_left = 0;
  int pending = -1;
  bool exhausted = false;
  bool active = false;
  RayState r;
  size_t slot = 0;

  while (true) {
    // ---- refill idle lanes from the current item's pool
    while (true) {
      const uint64_t idle = __ballot(!active);
      if (idle == 0) break;
      if (pool_left == 0) {
        if (pending >= 0 || exhausted) break;
        int it = 0;
        if (lane == 0) it = atomicAdd(bg.head, 1);
        // wave-uniform: the item, and so the brick, live in scalar registers
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
        if (it >= bg.n_items) {
          exhausted = true;
          break;
        }
        if (bg.item_count && lane == 0) atomicAdd(bg.item_count + it, 1);
        const BatchItem I = bg.items[it];
        if (I.cam != cur_cam || I.brick != cur_brick) {
          if (__ballot(active) != 0) {  // drain the current rays first
            pending = it;
            break;
          }
          cur_cam = I.cam;
          cur_brick = I.brick;
        }
        pool_item = it;
        pool_next = 0;
        pool_left = tp;
      }
      const int n_idle = __popcll(idle);
      const int take = min(n_idle, pool_left);
      const int rank = __popcll(idle & lt_mask);
      if (!active && rank < take) {
        const int pix = pool_next + rank;
        const BatchItem I = bg.items[pool_item];
        const CamG& cam = bg.cams[cur_cam];
        const int px = I.tx * bg.tile_w + pix % bg.tile_w;
        const int py = I.ty * bg.tile_h + pix / bg.tile_w;
        slot = (size_t)pool_item * tp + pix;
        bool hit = false;
        if (px < cam.W && py < cam.H) {
          double d[3];
          camera_ray(cam, px, py, d);
          hit = ray_start<T, WIDE, ISO>(sc, bg.bricks[cur_brick], cam.eye, d, r);
        }
        if (hit) {
          active = true;
        } else {
          bg.frag_rgba[slot] = make_float4(0.f, 0.f, 0.f, 0.f);
          bg.frag_depth[slot] = INFINITY;
          if (bg.slot_count) atomicAdd(bg.slot_count + slot, 1);
        }
      }
      pool_next += take;
      pool_left -= take;
    }
    // ---- nothing to march: switch to the pending item or finish
    if (__ballot(active) == 0) {
      if (pending >= 0) {
        const BatchItem I = bg.items[pending];
        cur_cam = I.cam;
        cur_brick = I.brick;
        pool_item = pending;
        pool_next = 0;
        pool_left = tp;
        pending = -1;
        continue;
      }
      if (exhausted) break;
      continue;
    }
    // ---- march a chunk of segments
    if (active) {
      // early return for a refill (fewer than half the lanes marching), only while
      // a refill can take rays
      const int min_lanes = (!exhausted && pending < 0) ? kRefillLanes : 0;
      if (ray_advance<T, SKIP, WIDE, ISO>(sc, bg.bricks[cur_brick], tfb, tfs, r, kChunk, min_lanes)) {
        bg.frag_rgba[slot] = make_float4(r.cr, r.cg, r.cb, 1.f - r.T);
        bg.frag_depth[slot] = (float)r.t_in;
        if (bg.slot_count) atomicAdd(bg.slot_count + slot, 1);
        active = false;
      }
    }
  }
}

// Per camera tile: composite the fragments of the items that cover it.  One wave
// per 64 pixels of a tile.
template <int KMAX>
__global__ __launch_bounds__(64) void tile_composite_kernel(BatchG bg, const int* __restrict__ tile_cam,
                                                            const int* __restrict__ tile_xy,
                                                            const int* __restrict__ tile_off,
                                                            const int* __restrict__ tile_items,
                                                            float4* const* __restrict__ out_rgba,
                                                            float* const* __restrict__ out_depth, int chunks) {
  __shared__ CompLDS<KMAX> s;
  const int g = blockIdx.x / chunks;
  const int q = blockIdx.x % chunks;
  const int lane = threadIdx.x;
  const int c = tile_cam[g];
  const CamG& cam = bg.cams[c];
  const int tp = bg.tile_w * bg.tile_h;
  const int pix = q * 64 + lane;
  const int px = tile_xy[2 * g] * bg.tile_w + pix % bg.tile_w;
  const int py = tile_xy[2 * g + 1] * bg.tile_h + pix / bg.tile_w;
  const bool live_px = pix < tp && px < cam.W && py < cam.H;
  const int k0 = tile_off[g];
  const int K = tile_off[g + 1] - k0;
  float4 col = make_float4(0.f, 0.f, 0.f, 0.f);
  float z = INFINITY;
  if (K > 0) {
    composite_wave<KMAX>(
        s, K, live_px, [&](int k) { return bg.frag_depth[(size_t)tile_items[k0 + k] * tp + pix]; },
        [&](int k) { return bg.frag_rgba[(size_t)tile_items[k0 + k] * tp + pix]; },
        [&](int k) { return bg.items[tile_items[k0 + k]].brick; }, col, z);
  }
  if (live_px) {
    const size_t p = (size_t)py * cam.W + px;
    out_rgba[c][p] = col;
    out_depth[c][p] = z;
  }
}

// Deep-frame target of the tile pass (dpr_render_deep): per pixel the count and
// the sorted fragments, layer-major (layer i of pixel p at i * P + p).
struct DeepOut {
  int* counts;
  float4* rgba;
  float* depth;
  int* ids;
  size_t P;
  int rank;
};

// Per camera tile: sort each pixel's fragments of the items covering the tile by
// (depth, brick) and write them as the pixel's deep-frame layers.  One wave per 64
// pixels of a tile; one camera.
template <int KMAX>
__global__ __launch_bounds__(64) void tile_deep_kernel(BatchG bg, const int* __restrict__ tile_xy,
                                                       const int* __restrict__ tile_off,
                                                       const int* __restrict__ tile_items, DeepOut dout,
                                                       int chunks) {
  __shared__ CompLDS<KMAX> s;
  const int g = blockIdx.x / chunks;
  const int q = blockIdx.x % chunks;
  const int lane = threadIdx.x;
  const CamG& cam = bg.cams[0];
  const int tp = bg.tile_w * bg.tile_h;
  const int pix = q * 64 + lane;
  const int px = tile_xy[2 * g] * bg.tile_w + pix % bg.tile_w;
  const int py = tile_xy[2 * g + 1] * bg.tile_h + pix / bg.tile_w;
  const bool live_px = pix < tp && px < cam.W && py < cam.H;
  const int k0 = tile_off[g];
  const int K = tile_off[g + 1] - k0;
  int n = 0;
  if (K > 0)
    n = sort_wave<KMAX>(
        s, K, live_px, [&](int k) { return bg.frag_depth[(size_t)tile_items[k0 + k] * tp + pix]; },
        [&](int k) { return bg.items[tile_items[k0 + k]].brick; });
  if (live_px) {
    const size_t p = (size_t)py * cam.W + px;
    dout.counts[p] = n;
    for (int i = 0; i < n; ++i) {
      const int k = s.lst[i][lane];
      const int item = tile_items[k0 + k];
      dout.rgba[(size_t)i * dout.P + p] = bg.frag_rgba[(size_t)item * tp + pix];
      dout.depth[(size_t)i * dout.P + p] = s.zs[k][lane];
      dout.ids[(size_t)i * dout.P + p] = dout.rank * 65536 + bg.items[item].brick;
    }
  }
}

struct BatchState {
  // key
  std::vector<dpr_camera> cams;
  std::vector<dpr_frame> outs;
  std::vector<const void*> out_ptrs;
  int tile_w = 0, tile_h = 0;
  int brick_sel = -1;  // the one brick rendered (dpr_render_partial), or -1 for all
  uint64_t geo_version = 0;
  bool skip = true;
  // deep-frame target (dpr_render_deep) instead of flat frames, and its buffers
  dpr_deep_frame deep = nullptr;
  const void* deep_ptrs[4] = {nullptr, nullptr, nullptr, nullptr};
  int deep_rank = -1;
  // brick views last uploaded to d_bricks, and the scene arguments and TF table
  // baked into the captured graph
  std::vector<BrickG> h_bricks;
  SceneG cap_scene{};
  const float4* cap_tf = nullptr;
  // device data
  CamG* d_cams = nullptr;
  BrickG* d_bricks = nullptr;
  BatchItem* d_items = nullptr;
  int* d_tile_cam = nullptr;
  int* d_tile_xy = nullptr;
  int* d_tile_off = nullptr;
  int* d_tile_items = nullptr;
  float4** d_out_rgba = nullptr;
  float** d_out_depth = nullptr;
  float4* frag_rgba = nullptr;
  float* frag_depth = nullptr;
  int* head = nullptr;
  int* item_count = nullptr;  // queue-coverage counters, allocated on first use
  int* slot_count = nullptr;
  bool counted = false;       // the last render counted
  int n_items = 0, n_tiles = 0, max_k = 0;
  int grid[2] = {0, 0};  // persistent grid of the march kernel without / with iso-surface
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // before march, after march, after composite
  bool timed = false;                               // events were recorded by the last render
  // plain per-brick path
  std::vector<dpr_frame> plain_parts;

  void free_device() {
    for (void* p : {(void*)d_cams, (void*)d_bricks, (void*)d_items, (void*)d_tile_cam, (void*)d_tile_xy,
                    (void*)d_tile_off, (void*)d_tile_items, (void*)d_out_rgba, (void*)d_out_depth,
                    (void*)frag_rgba, (void*)frag_depth, (void*)head, (void*)item_count, (void*)slot_count})
      dev_free(p);
    d_cams = nullptr;
    d_bricks = nullptr;
    d_items = nullptr;
    d_tile_cam = d_tile_xy = d_tile_off = d_tile_items = nullptr;
    d_out_rgba = nullptr;
    d_out_depth = nullptr;
    frag_rgba = nullptr;
    frag_depth = nullptr;
    head = nullptr;
    item_count = slot_count = nullptr;
    counted = false;
    drop_graph();
  }
  // 64-bit offsets for every brick if any brick the launch reads needs them
  bool wide() const {
    if (brick_sel >= 0) return brick_sel < (int)h_bricks.size() && h_bricks[brick_sel].wide;
    for (const auto& g : h_bricks)
      if (g.wide) return true;
    return false;
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~BatchState() {
    free_device();
    for (auto f : plain_parts) dpr_frame_release(f);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

void batch_state_free(BatchState* s) { delete s; }

// Length of the chord that the ray through pixel (x, y) cuts from the box [lo, hi]
// (0 on a miss): the work estimate used to order a brick's tiles.
static double chord_length(const CamG& c, double x, double y, const double lo[3], const double hi[3]) {
  const double sx = (2.0 * (x + 0.5) / c.W - 1.0) * c.sx, sy = (1.0 - 2.0 * (y + 0.5) / c.H) * c.sy;
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = c.f[a] + sx * c.r[a] + sy * c.u[a];
  const double inv = 1.0 / std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double tn = 0.0, tf = 1e300;
  for (int a = 0; a < 3; ++a) {
    const double da = d[a] * inv;
    if (da == 0.0) {
      if (c.eye[a] < lo[a] || c.eye[a] > hi[a]) return 0.0;
      continue;
    }
    const double t0 = (lo[a] - c.eye[a]) / da, t1 = (hi[a] - c.eye[a]) / da;
    tn = std::max(tn, std::min(t0, t1));
    tf = std::min(tf, std::max(t0, t1));
  }
  return tf > tn ? tf - tn : 0.0;
}

// Conservative screen rectangle (pixel indices, inclusive) of a box's projection.
static void brick_screen_rect(const CamG& c, const double lo[3], const double hi[3], int& x0, int& y0, int& x1,
                              int& y1) {
  double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300;
  for (int i = 0; i < 8; ++i) {
    double p[3] = {(i & 1) ? hi[0] : lo[0], (i & 2) ? hi[1] : lo[1], (i & 4) ? hi[2] : lo[2]};
    double v[3] = {p[0] - c.eye[0], p[1] - c.eye[1], p[2] - c.eye[2]};
    double z = v[0] * c.f[0] + v[1] * c.f[1] + v[2] * c.f[2];
    if (!(z > 1e-9)) {  // a corner at or behind the eye: take the whole screen
      x0 = 0;
      y0 = 0;
      x1 = c.W - 1;
      y1 = c.H - 1;
      return;
    }
    double x = (v[0] * c.r[0] + v[1] * c.r[1] + v[2] * c.r[2]) / z;
    double y = (v[0] * c.u[0] + v[1] * c.u[1] + v[2] * c.u[2]) / z;
    double px = (x / c.sx + 1.0) * 0.5 * c.W - 0.5;
    double py = (1.0 - y / c.sy) * 0.5 * c.H - 0.5;
    mnx = std::min(mnx, px);
    mxx = std::max(mxx, px);
    mny = std::min(mny, py);
    mxy = std::max(mxy, py);
  }
  x0 = (int)std::max(0.0, std::floor(mnx) - 1.0);
  y0 = (int)std::max(0.0, std::floor(mny) - 1.0);
  x1 = (int)std::min((double)c.W - 1, std::ceil(mxx) + 1.0);
  y1 = (int)std::min((double)c.H - 1, std::ceil(mxy) + 1.0);
}

template <typename V>
static dpr_status upload(V** dst, const std::vector<V>& src, hipStream_t st, const char* what) {
  dpr_status s = dev_alloc((void**)dst, std::max<size_t>(1, src.size()) * sizeof(V), what);
  if (s != DPR_OK) return s;
  if (!src.empty()) DPR_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice, st));
  DPR_HIP(hipStreamSynchronize(st));
  return DPR_OK;
}

template <typename T, bool SKIP, bool ISO>
static const void* march_fn_t(bool wide) {
  return wide ? (const void*)batch_march_kernel<T, SKIP, true, ISO>
              : (const void*)batch_march_kernel<T, SKIP, false, ISO>;
}

template <typename T, bool SKIP>
static const void* march_fn_s(bool wide, bool iso) {
  return iso ? march_fn_t<T, SKIP, true>(wide) : march_fn_t<T, SKIP, false>(wide);
}

static const void* march_fn(bool f16, bool skip, bool wide, bool iso) {
  if (f16) return skip ? march_fn_s<__half, true>(wide, iso) : march_fn_s<__half, false>(wide, iso);
  return skip ? march_fn_s<float, true>(wide, iso) : march_fn_s<float, false>(wide, iso);
}

static hipError_t enqueue_batch(dpr_world w, BatchState* b, hipStream_t st, bool timed, bool count = false) {
  SceneG sc = make_scene(w);
  BatchG g{};
  g.cams = b->d_cams;
  g.bricks = b->d_bricks;
  g.items = b->d_items;
  g.n_items = b->n_items;
  g.tile_w = b->tile_w;
  g.tile_h = b->tile_h;
  g.frag_rgba = b->frag_rgba;
  g.frag_depth = b->frag_depth;
  g.head = b->head;
  if (count) {
    const size_t slots = (size_t)b->n_items * b->tile_w * b->tile_h;
    g.item_count = b->item_count;
    g.slot_count = b->slot_count;
    hipLaunchKernelGGL(zero_counts_kernel, dim3(256), dim3(256), 0, st, b->item_count, (size_t)b->n_items);
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1024), dim3(256), 0, st, b->slot_count, slots);
  }
  const bool f16 = w->bricks[b->brick_sel >= 0 ? b->brick_sel : 0].dtype == DPR_F16;
  size_t lds = 2 * sizeof(float4) * (size_t)sc.ntf;
  hipLaunchKernelGGL(reset_head_kernel, dim3(1), dim3(1), 0, st, b->head);
  if (timed) (void)hipEventRecord(b->ev[0], st);
  const int iso = sc.iso_on ? 1 : 0;
  const void* fn = march_fn(f16, b->skip, b->wide(), iso);
  void* args[] = {(void*)&sc, (void*)&g, (void*)&w->tf_dev};
  const hipError_t le = hipLaunchKernel(fn, dim3(b->grid[iso]), dim3(256), args, lds, st);
  if (le != hipSuccess) return le;
  if (timed) (void)hipEventRecord(b->ev[1], st);
  const int tp = b->tile_w * b->tile_h;
  const int chunks = (tp + 63) / 64;
  dim3 cgrid((unsigned)b->n_tiles * chunks);
  if (b->deep) {
    const dpr_deep_frame d = b->deep;
    DeepOut dout{d->counts, d->rgba, d->depth, d->ids, (size_t)d->w * d->h, b->deep_rank};
    if (b->max_k <= 16)
      hipLaunchKernelGGL(tile_deep_kernel<16>, cgrid, dim3(64), 0, st, g, b->d_tile_xy, b->d_tile_off,
                         b->d_tile_items, dout, chunks);
    else if (b->max_k <= 64)
      hipLaunchKernelGGL(tile_deep_kernel<64>, cgrid, dim3(64), 0, st, g, b->d_tile_xy, b->d_tile_off,
                         b->d_tile_items, dout, chunks);
    else
      hipLaunchKernelGGL(tile_deep_kernel<256>, cgrid, dim3(64), 0, st, g, b->d_tile_xy, b->d_tile_off,
                         b->d_tile_items, dout, chunks);
  } else {
    if (b->max_k <= 16)
      hipLaunchKernelGGL(tile_composite_kernel<16>, cgrid, dim3(64), 0, st, g, b->d_tile_cam, b->d_tile_xy,
                         b->d_tile_off, b->d_tile_items, b->d_out_rgba, b->d_out_depth, chunks);
    else if (b->max_k <= 64)
      hipLaunchKernelGGL(tile_composite_kernel<64>, cgrid, dim3(64), 0, st, g, b->d_tile_cam, b->d_tile_xy,
                         b->d_tile_off, b->d_tile_items, b->d_out_rgba, b->d_out_depth, chunks);
    else
      hipLaunchKernelGGL(tile_composite_kernel<256>, cgrid, dim3(64), 0, st, g, b->d_tile_cam, b->d_tile_xy,
                         b->d_tile_off, b->d_tile_items, b->d_out_rgba, b->d_out_depth, chunks);
  }
  if (timed) (void)hipEventRecord(b->ev[2], st);
  return hipGetLastError();
}

// (Re)build the item queue, tile lists and fragment storage for these cameras.
static dpr_status build_batch(dpr_world w, BatchState* b, const dpr_camera* cams, int n, const dpr_frame* outs,
                              int tw, int th, int brick_sel) {
  hipStream_t st = w->dev->stream;
  DPR_HIP(hipStreamSynchronize(st));
  b->free_device();
  b->cams.assign(cams, cams + n);
  b->outs.assign(outs, outs + n);
  b->out_ptrs.clear();
  for (int c = 0; c < n; ++c) {
    b->out_ptrs.push_back(outs[c] ? outs[c]->rgba : nullptr);
    b->out_ptrs.push_back(outs[c] ? outs[c]->depth : nullptr);
  }
  b->tile_w = tw;
  b->tile_h = th;
  b->brick_sel = brick_sel;
  b->geo_version = w->geo_version;
  b->skip = !(w->params.flags & DPR_FLAG_NO_SKIP);
  const SceneG sc = make_scene(w);
  std::vector<CamG> cg(n);
  for (int c = 0; c < n; ++c) cg[c] = make_cam(cams[c]);
  std::vector<BrickG> bg;
  for (const auto& br : w->bricks) bg.push_back(br.device_view(b->skip, w->params.flags & DPR_FLAG_WIDE_OFFSETS));
  // items grouped by (camera, brick), so consecutive pops share a brick; inside a
  // group, tiles by decreasing chord of their centre ray through the brick, so the
  // longest rays start first and the rays still marching when a group (or the
  // whole queue) runs out are short ones
  std::vector<BatchItem> items;
  std::vector<int> tiles_x(n), tile_base(n + 1, 0);
  for (int c = 0; c < n; ++c) {
    tiles_x[c] = (cams[c].width + tw - 1) / tw;
    int ty = (cams[c].height + th - 1) / th;
    tile_base[c + 1] = tile_base[c] + tiles_x[c] * ty;
  }
  std::vector<std::vector<int>> per_tile(tile_base[n]);
  for (int c = 0; c < n; ++c) {
    for (int k = 0; k < (int)w->bricks.size(); ++k) {
      if (brick_sel >= 0 && k != brick_sel) continue;
      const Brick& br = w->bricks[k];
      double lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = br.olo[a] * sc.h;
        hi[a] = br.ohi[a] * sc.h;
      }
      int x0, y0, x1, y1;
      brick_screen_rect(cg[c], lo, hi, x0, y0, x1, y1);
      if (x1 < x0 || y1 < y0) continue;
      std::vector<std::pair<double, BatchItem>> grp;
      for (int ty = y0 / th; ty <= y1 / th; ++ty)
        for (int tx = x0 / tw; tx <= x1 / tw; ++tx)
          grp.push_back({chord_length(cg[c], tx * tw + 0.5 * (tw - 1), ty * th + 0.5 * (th - 1), lo, hi),
                         BatchItem{c, k, tx, ty}});
      std::stable_sort(grp.begin(), grp.end(),
                       [](const std::pair<double, BatchItem>& a, const std::pair<double, BatchItem>& b2) {
                         return a.first > b2.first;
                       });
      for (const auto& e : grp) {
        per_tile[tile_base[c] + e.second.ty * tiles_x[c] + e.second.tx].push_back((int)items.size());
        items.push_back(e.second);
      }
    }
  }
  std::vector<int> tile_cam(tile_base[n]), tile_xy(2 * (size_t)tile_base[n]), tile_off(tile_base[n] + 1, 0),
      tile_items;
  int max_k = 1;
  for (int c = 0; c < n; ++c)
    for (int t = tile_base[c]; t < tile_base[c + 1]; ++t) {
      int local = t - tile_base[c];
      tile_cam[t] = c;
      tile_xy[2 * (size_t)t] = local % tiles_x[c];
      tile_xy[2 * (size_t)t + 1] = local / tiles_x[c];
      tile_off[t + 1] = tile_off[t] + (int)per_tile[t].size();
      max_k = std::max(max_k, (int)per_tile[t].size());
      tile_items.insert(tile_items.end(), per_tile[t].begin(), per_tile[t].end());
    }
  if (max_k > kMaxFrags) return fail(DPR_ERR_UNSUPPORTED, "dpr_render_batch: %d bricks cover one tile", max_k);
  b->n_items = (int)items.size();
  b->n_tiles = tile_base[n];
  b->max_k = max_k;
  std::vector<float4*> orgba(n);
  std::vector<float*> odepth(n);
  for (int c = 0; c < n; ++c) {
    orgba[c] = outs[c] ? (float4*)outs[c]->rgba : nullptr;
    odepth[c] = outs[c] ? outs[c]->depth : nullptr;
  }
  dpr_status s;
  if ((s = upload(&b->d_cams, cg, st, "batch cameras")) != DPR_OK) return s;
  if ((s = upload(&b->d_bricks, bg, st, "batch bricks")) != DPR_OK) return s;
  b->h_bricks = bg;
  if ((s = upload(&b->d_items, items, st, "batch items")) != DPR_OK) return s;
  if ((s = upload(&b->d_tile_cam, tile_cam, st, "batch tile cameras")) != DPR_OK) return s;
  if ((s = upload(&b->d_tile_xy, tile_xy, st, "batch tile coordinates")) != DPR_OK) return s;
  if ((s = upload(&b->d_tile_off, tile_off, st, "batch tile offsets")) != DPR_OK) return s;
  if ((s = upload(&b->d_tile_items, tile_items, st, "batch tile items")) != DPR_OK) return s;
  if ((s = upload(&b->d_out_rgba, orgba, st, "batch outputs")) != DPR_OK) return s;
  if ((s = upload(&b->d_out_depth, odepth, st, "batch outputs")) != DPR_OK) return s;
  size_t frags = std::max<size_t>(1, (size_t)b->n_items * tw * th);
  if ((s = dev_alloc((void**)&b->frag_rgba, frags * sizeof(float4), "batch fragments")) != DPR_OK) return s;
  if ((s = dev_alloc((void**)&b->frag_depth, frags * sizeof(float), "batch fragment depths")) != DPR_OK) return s;
  if ((s = dev_alloc((void**)&b->head, sizeof(int), "batch queue head")) != DPR_OK) return s;
  for (auto& e : b->ev)
    if (!e) DPR_HIP(hipEventCreate(&e));
  // persistent grid: as many 256-thread workgroups as fit on the GPU at once
  const bool f16 = w->bricks[brick_sel >= 0 ? brick_sel : 0].dtype == DPR_F16;
  size_t lds = 2 * sizeof(float4) * (size_t)sc.ntf;
  for (int iso = 0; iso < 2; ++iso) {
    int per_cu = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, march_fn(f16, b->skip, b->wide(), iso), 256, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    b->grid[iso] = w->dev->cu_count * per_cu;
  }
  return DPR_OK;
}

static dpr_status capture_graph(dpr_world w, BatchState* b) {
  if (!b->cap) DPR_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  DPR_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_batch(w, b, b->cap, false);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e, "dpr_render_batch: capture");
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  b->graph = g;
  DPR_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  b->cap_scene = make_scene(w);
  b->cap_tf = w->tf_dev;
  return DPR_OK;
}

// The item lists depend only on geometry (bricks, cameras, tile shape); data
// recommits and transfer-function changes only touch the brick views (device
// pointers, macrocell grids) and the scene arguments, which are refreshed here
// without rebuilding: brick views are re-uploaded when they changed, and the
// captured graph is dropped when an argument baked into it changed.
static dpr_status refresh_batch(dpr_world w, BatchState* b) {
  std::vector<BrickG> bg;
  for (const auto& br : w->bricks) bg.push_back(br.device_view(b->skip, w->params.flags & DPR_FLAG_WIDE_OFFSETS));
  if (bg.size() != b->h_bricks.size() || memcmp(bg.data(), b->h_bricks.data(), bg.size() * sizeof(BrickG)) != 0) {
    hipStream_t st = w->dev->stream;
    DPR_HIP(hipStreamSynchronize(st));
    b->drop_graph();
    DPR_HIP(hipMemcpyAsync(b->d_bricks, bg.data(), bg.size() * sizeof(BrickG), hipMemcpyHostToDevice, st));
    DPR_HIP(hipStreamSynchronize(st));
    b->h_bricks = bg;
  }
  if (b->exec) {
    const SceneG sc = make_scene(w);
    if (memcmp(&sc, &b->cap_scene, sizeof(SceneG)) != 0 || b->cap_tf != w->tf_dev) {
      DPR_HIP(hipStreamSynchronize(w->dev->stream));
      b->drop_graph();
    }
  }
  return DPR_OK;
}

static void deep_key(dpr_deep_frame d, const void* ptrs[4]) {
  ptrs[0] = d ? d->counts : nullptr;
  ptrs[1] = d ? d->rgba : nullptr;
  ptrs[2] = d ? d->depth : nullptr;
  ptrs[3] = d ? d->ids : nullptr;
}

static bool same_key(const BatchState* b, dpr_world w, const dpr_camera* cams, int n, const dpr_frame* outs, int tw,
                     int th, dpr_deep_frame deep, int rank, int brick_sel) {
  if (!b || b->tile_w != tw || b->tile_h != th || (int)b->cams.size() != n || b->brick_sel != brick_sel) return false;
  const void* dp[4];
  deep_key(deep, dp);
  if (b->deep != deep || b->deep_rank != rank || memcmp(b->deep_ptrs, dp, sizeof(dp)) != 0) return false;
  if (b->geo_version != w->geo_version || b->skip != !(w->params.flags & DPR_FLAG_NO_SKIP)) return false;
  if (memcmp(b->cams.data(), cams, n * sizeof(dpr_camera)) != 0) return false;
  for (int c = 0; c < n; ++c)
    if (b->outs[c] != outs[c] || (outs[c] && (b->out_ptrs[2 * c] != outs[c]->rgba ||
                                              b->out_ptrs[2 * c + 1] != outs[c]->depth)))
      return false;
  return b->d_items != nullptr;
}

static dpr_status check_batch_args(dpr_world w, const dpr_camera* cams, int n, const dpr_frame* outs) {
  if (!w || !cams || !outs) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_batch: NULL argument");
  if (n < 1) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_batch: n = %d", n);
  if (!w->committed) return fail(DPR_ERR_INVALID_STATE, "dpr_render_batch: world not committed");
  if (!w->tf_set) return fail(DPR_ERR_INVALID_STATE, "dpr_render_batch: no transfer function set");
  for (int c = 0; c < n; ++c) {
    dpr_status s = check_camera(&cams[c]);
    if (s != DPR_OK) return s;
    if (!outs[c]) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_batch: frame %d is NULL", c);
    if (outs[c]->w != cams[c].width || outs[c]->h != cams[c].height)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_batch: frame %d size differs from its camera", c);
    if (outs[c]->dev != w->dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_batch: frame of another device");
  }
  for (const auto& b : w->bricks)
    if (b.dtype != w->bricks[0].dtype)
      return fail(DPR_ERR_UNSUPPORTED, "dpr_render_batch: bricks of mixed dtypes");
  if ((int)w->bricks.size() > kMaxFrags)
    return fail(DPR_ERR_UNSUPPORTED, "dpr_render_batch: more than %d bricks", kMaxFrags);
  return DPR_OK;
}

// Baseline: per camera, one plain launch per brick into full partial frames, then
// the K-frame compositor.
static dpr_status render_plain(dpr_world w, const dpr_camera* cams, int n, dpr_frame* outs) {
  if (!w->batch) w->batch = new BatchState;
  BatchState* b = w->batch;
  const int K = (int)w->bricks.size();
  const bool skip = !(w->params.flags & DPR_FLAG_NO_SKIP);
  SceneG sc = make_scene(w);
  std::vector<int32_t> ids(K);
  std::iota(ids.begin(), ids.end(), 0);
  for (int c = 0; c < n; ++c) {
    bool resize = (int)b->plain_parts.size() != K;
    for (auto f : b->plain_parts) resize |= f->w != cams[c].width || f->h != cams[c].height;
    if (resize) {
      DPR_HIP(hipStreamSynchronize(w->dev->stream));
      for (auto f : b->plain_parts) dpr_frame_release(f);
      b->plain_parts.clear();
      for (int i = 0; i < K; ++i) {
        dpr_frame f = nullptr;
        dpr_status s = dpr_frame_create(w->dev, cams[c].width, cams[c].height, &f);
        if (s != DPR_OK) return s;
        b->plain_parts.push_back(f);
      }
    }
    CamG cg = make_cam(cams[c]);
    for (int i = 0; i < K; ++i) {
      const Brick& br = w->bricks[i];
      DPR_HIP(launch_march(sc, br.device_view(skip, w->params.flags & DPR_FLAG_WIDE_OFFSETS), cg, w->tf_dev, br.dtype == DPR_F16, skip,
                           (float4*)b->plain_parts[i]->rgba, b->plain_parts[i]->depth, nullptr, w->dev->stream));
    }
    dpr_status s = composite_frames(w->dev, b->plain_parts.data(), ids.data(), K, outs[c]);
    if (s != DPR_OK) return s;
  }
  return DPR_OK;
}

static dpr_status render_batch_state(dpr_world w, BatchState* b, const dpr_camera* cams, int n, dpr_frame* outs,
                                     uint32_t flags, int tw, int th, dpr_deep_frame deep, int rank, int brick_sel) {
  dpr_status s = ensure_majorants(w);
  if (s != DPR_OK) return s;
  if (!same_key(b, w, cams, n, outs, tw, th, deep, rank, brick_sel)) {
    s = build_batch(w, b, cams, n, outs, tw, th, brick_sel);
    if (s != DPR_OK) return s;
    b->deep = deep;
    b->deep_rank = rank;
    deep_key(deep, b->deep_ptrs);
  } else {
    s = refresh_batch(w, b);
    if (s != DPR_OK) return s;
  }
  w->last_batch = b;
  b->counted = false;
  if (flags & DPR_FLAG_QUEUE_COVERAGE) {
    if (!b->item_count) {
      const size_t slots = (size_t)b->n_items * b->tile_w * b->tile_h;
      s = dev_alloc((void**)&b->item_count, std::max<size_t>(1, b->n_items) * sizeof(int), "queue coverage counters");
      if (s != DPR_OK) return s;
      s = dev_alloc((void**)&b->slot_count, std::max<size_t>(1, slots) * sizeof(int), "queue coverage counters");
      if (s != DPR_OK) return s;
    }
    DPR_HIP(enqueue_batch(w, b, w->dev->stream, true, true));
    b->timed = true;
    b->counted = true;
    return DPR_OK;
  }
  if (flags & DPR_FLAG_NO_GRAPH) {
    DPR_HIP(enqueue_batch(w, b, w->dev->stream, true));
    b->timed = true;
    return DPR_OK;
  }
  if (!b->exec) {
    s = capture_graph(w, b);
    if (s != DPR_OK) return s;
  }
  DPR_HIP(hipGraphLaunch(b->exec, w->dev->stream));
  b->timed = false;
  return DPR_OK;
}

static dpr_status render_batch_tiled(dpr_world w, const dpr_camera* cams, int n, dpr_frame* outs, uint32_t flags,
                                     int tw, int th, dpr_deep_frame deep = nullptr, int rank = -1) {
  if (!w->batch) w->batch = new BatchState;
  return render_batch_state(w, w->batch, cams, n, outs, flags, tw, th, deep, rank, -1);
}

// render-parameter flags the batched paths take from the world
constexpr uint32_t kBatchFlags = DPR_FLAG_NO_GRAPH | DPR_FLAG_QUEUE_COVERAGE;

// One brick's partial frame through the persistent kernel: items of that brick
// only (one cached state per brick), every camera tile written by the tile pass
// (tiles the brick does not cover come out empty).
dpr_status render_partial_batched(dpr_world w, int id, dpr_frame out) {
  if ((int)w->partial_batch.size() < (int)w->bricks.size()) w->partial_batch.resize(w->bricks.size(), nullptr);
  if (!w->partial_batch[id]) w->partial_batch[id] = new BatchState;
  return render_batch_state(w, w->partial_batch[id], &w->cam, 1, &out, w->params.flags & kBatchFlags,
                            w->batch_tile_w, w->batch_tile_h, nullptr, -1, id);
}

dpr_status render_frame_batched(dpr_world w, dpr_frame out) {
  return render_batch_tiled(w, &w->cam, 1, &out, w->params.flags & kBatchFlags, w->batch_tile_w,
                            w->batch_tile_h);
}

static dpr_status render_deep(dpr_world w, int rank, dpr_deep_frame out) {
  dpr_frame none = nullptr;
  dpr_status s = render_batch_tiled(w, &w->cam, 1, &none, w->params.flags & kBatchFlags, w->batch_tile_w,
                                    w->batch_tile_h, out, rank);
  if (s != DPR_OK) return s;
  out->rank = rank;
  return DPR_OK;
}

}  // namespace dpr

using namespace dpr;

extern "C" {

dpr_status dpr_render_batch(dpr_world w, const dpr_camera* cams, int32_t n, dpr_frame* outs, uint32_t flags) {
  dpr_status s = check_batch_args(w, cams, n, outs);
  if (s != DPR_OK) return s;
  if (flags & DPR_FLAG_PLAIN) {
    s = ensure_majorants(w);
    if (s != DPR_OK) return s;
    return render_plain(w, cams, n, outs);
  }
  return render_batch_tiled(w, cams, n, outs, flags, w->batch_tile_w, w->batch_tile_h);
}

dpr_status dpr_render_deep(dpr_world w, int32_t rank, dpr_deep_frame out) {
  if (!w || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_deep: NULL argument");
  if (!w->committed) return fail(DPR_ERR_INVALID_STATE, "dpr_render_deep: world not committed");
  if (!w->tf_set) return fail(DPR_ERR_INVALID_STATE, "dpr_render_deep: no transfer function set");
  if (!w->cam_set) return fail(DPR_ERR_INVALID_STATE, "dpr_render_deep: no camera set");
  if (rank < 0 || rank >= 32768) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_deep: rank %d", rank);
  if (out->dev != w->dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_deep: frame of another device");
  if (out->w != w->cam.width || out->h != w->cam.height)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_deep: frame %dx%d != camera %dx%d", out->w, out->h,
                w->cam.width, w->cam.height);
  if (out->cap < (int)w->bricks.size())
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_deep: capacity %d < %d bricks", out->cap,
                (int)w->bricks.size());
  for (const auto& b : w->bricks)
    if (b.dtype != w->bricks[0].dtype) return fail(DPR_ERR_UNSUPPORTED, "dpr_render_deep: bricks of mixed dtypes");
  return render_deep(w, rank, out);
}

dpr_status dpr_batch_timings(dpr_world w, float* march_ms, float* composite_ms) {
  if (!w) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_batch_timings: NULL world");
  BatchState* b = w->last_batch;
  if (!b || !b->timed || !b->ev[0])
    return fail(DPR_ERR_INVALID_STATE, "dpr_batch_timings: the last batched render was not enqueued directly");
  DPR_HIP(hipEventSynchronize(b->ev[2]));
  float a = 0.f, c = 0.f;
  DPR_HIP(hipEventElapsedTime(&a, b->ev[0], b->ev[1]));
  DPR_HIP(hipEventElapsedTime(&c, b->ev[1], b->ev[2]));
  if (march_ms) *march_ms = a;
  if (composite_ms) *composite_ms = c;
  return DPR_OK;
}

dpr_status dpr_batch_coverage(dpr_world w, int64_t out[4]) {
  if (!w || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_batch_coverage: NULL argument");
  BatchState* b = w->last_batch;
  if (!b || !b->counted)
    return fail(DPR_ERR_INVALID_STATE, "dpr_batch_coverage: the last batched render did not count its queue");
  const size_t slots = (size_t)b->n_items * b->tile_w * b->tile_h;
  std::vector<int> items(b->n_items), marks(slots);
  DPR_HIP(hipStreamSynchronize(w->dev->stream));
  if (b->n_items > 0) {
    DPR_HIP(hipMemcpy(items.data(), b->item_count, items.size() * sizeof(int), hipMemcpyDeviceToHost));
    DPR_HIP(hipMemcpy(marks.data(), b->slot_count, marks.size() * sizeof(int), hipMemcpyDeviceToHost));
  }
  out[0] = (int64_t)items.size();
  out[1] = std::count(items.begin(), items.end(), 1);
  out[2] = (int64_t)marks.size();
  out[3] = std::count(marks.begin(), marks.end(), 1);
  return DPR_OK;
}

dpr_status dpr_set_batch_tile(dpr_world w, int32_t tw, int32_t th) {
  if (!w) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_batch_tile: NULL world");
  if (tw < 1 || th < 1 || (tw * th) % 64 != 0 || tw * th > 1024)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_batch_tile: %dx%d is not a multiple of 64 pixels <= 1024", tw, th);
  w->batch_tile_w = tw;
  w->batch_tile_h = th;
  return DPR_OK;
}

dpr_status dpr_autotune_batch(dpr_world w, const dpr_camera* cams, int32_t n, dpr_frame* outs, int32_t* tw_out,
                              int32_t* th_out) {
  dpr_status s = check_batch_args(w, cams, n, outs);
  if (s != DPR_OK) return s;
  // the persisted choice for this device and shape of work, if any
  const char* cache = getenv("DPR_TUNE_CACHE");
  std::string key;
  if (cache && cache[0]) {
    const Brick& b0 = w->bricks[0];
    key = "gfx950 cu" + std::to_string(w->dev->cu_count) +
          (b0.dtype == DPR_F16 ? (b0.half16 ? " f16-2byte" : " f16-pairs") : " f32") + " bricks";
    for (const auto& br : w->bricks)
      key += " " + std::to_string(br.sdim[0]) + "x" + std::to_string(br.sdim[1]) + "x" + std::to_string(br.sdim[2]);
    key += " cameras";
    for (int c = 0; c < n; ++c) key += " " + std::to_string(cams[c].width) + "x" + std::to_string(cams[c].height);
    char prm[128];
    snprintf(prm, sizeof prm, " step %g ert %g mc %d flags %u", w->params.step_voxels, w->params.ert_threshold,
             w->params.macrocell_cells, w->params.flags & (DPR_FLAG_NO_SKIP | DPR_FLAG_WIDE_OFFSETS));
    key += prm;
    int32_t found = 0, cw = 0, ch = 0;
    s = dpr_tune_cache_lookup(cache, key.c_str(), &found, &cw, &ch);
    if (s != DPR_OK) return s;
    if (found && dpr_set_batch_tile(w, cw, ch) == DPR_OK) {
      s = render_batch_tiled(w, cams, n, outs, 0, cw, ch);  // leave the chosen shape built
      if (s != DPR_OK) return s;
      if (tw_out) *tw_out = cw;
      if (th_out) *th_out = ch;
      return DPR_OK;
    }
  }
  static const int cand[][2] = {{8, 8}, {16, 8}, {16, 16}, {32, 16}, {32, 32}};
  hipEvent_t e0, e1;
  DPR_HIP(hipEventCreate(&e0));
  DPR_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bw = w->batch_tile_w, bh = w->batch_tile_h;
  for (const auto& c : cand) {
    s = render_batch_tiled(w, cams, n, outs, 0, c[0], c[1]);  // build + capture + warm-up
    if (s != DPR_OK) break;
    DPR_HIP(hipEventRecord(e0, w->dev->stream));
    for (int r = 0; r < 3; ++r) {
      s = render_batch_tiled(w, cams, n, outs, 0, c[0], c[1]);
      if (s != DPR_OK) break;
    }
    DPR_HIP(hipEventRecord(e1, w->dev->stream));
    DPR_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    DPR_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (log_enabled()) fprintf(stderr, "[dpr] autotune tile %dx%d: %.3f ms\n", c[0], c[1], ms / 3);
    if (ms < best) {
      best = ms;
      bw = c[0];
      bh = c[1];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != DPR_OK) return s;
  w->batch_tile_w = bw;
  w->batch_tile_h = bh;
  s = render_batch_tiled(w, cams, n, outs, 0, bw, bh);  // leave the chosen shape built
  if (s != DPR_OK) return s;
  if (!key.empty()) {
    s = dpr_tune_cache_store(cache, key.c_str(), bw, bh);
    if (s != DPR_OK) return s;
  }
  if (tw_out) *tw_out = bw;
  if (th_out) *th_out = bh;
  return DPR_OK;
}

}  // extern "C"
