// C ABI implementation: devices, worlds, bricks, frames, validation and the
// per-brick render / composite entry points.
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>

#include "runtime.hpp"

namespace dpr {

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  if (log_enabled()) fprintf(stderr, "[dpr] %s\n", buf);
}

dpr_status fail(dpr_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  if (log_enabled()) fprintf(stderr, "[dpr] %s\n", buf);
  return st;
}

dpr_status hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();  // clear the thread's HIP error so it does not surface in unrelated calls
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(DPR_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
  return fail(DPR_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool log_enabled() {
  static int on = -1;
  if (on < 0) {
    const char* s = getenv("DPR_LOG");
    on = (s && s[0] == '1') ? 1 : 0;
  }
  return on == 1;
}

static std::atomic<long> g_alloc_count{0};  // allocations attempted
static std::atomic<long> g_alloc_live{0};   // allocations not yet freed

static bool injected_failure(long n) {
  const char* fi = getenv("DPR_FAULT_INJECT");
  return fi && strncmp(fi, "alloc:", 6) == 0 && atol(fi + 6) == n;
}

dpr_status dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  const long n = ++g_alloc_count;
  if (injected_failure(n)) return fail(DPR_ERR_OUT_OF_MEMORY, "%s: injected allocation failure (allocation %ld)", what, n);
  hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(DPR_ERR_OUT_OF_MEMORY, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  ++g_alloc_live;
  return DPR_OK;
}

void dev_free(void* p) {
  if (!p) return;
  (void)hipFree(p);
  --g_alloc_live;
}

dpr_status host_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  const long n = ++g_alloc_count;
  if (injected_failure(n)) return fail(DPR_ERR_OUT_OF_MEMORY, "%s: injected allocation failure (allocation %ld)", what, n);
  hipError_t e = hipHostMalloc(p, bytes ? bytes : 1, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(DPR_ERR_OUT_OF_MEMORY, "%s: hipHostMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  ++g_alloc_live;
  return DPR_OK;
}

void host_free(void* p) {
  if (!p) return;
  (void)hipHostFree(p);
  --g_alloc_live;
}

// ---------------------------------------------------------------- geometry helpers
CamG make_cam(const dpr_camera& c) {
  CamG g{};
  double f[3] = {c.center[0] - c.eye[0], c.center[1] - c.eye[1], c.center[2] - c.eye[2]};
  double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double& v : f) v /= fn;
  double r[3] = {f[1] * c.up[2] - f[2] * c.up[1], f[2] * c.up[0] - f[0] * c.up[2], f[0] * c.up[1] - f[1] * c.up[0]};
  double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double& v : r) v /= rn;
  double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  for (int a = 0; a < 3; ++a) {
    g.eye[a] = c.eye[a];
    g.f[a] = f[a];
    g.r[a] = r[a];
    g.u[a] = u[a];
  }
  double th = std::tan(c.fovy_deg * M_PI / 360.0);
  g.sy = th;
  g.sx = th * (double)c.width / (double)c.height;
  g.W = c.width;
  g.H = c.height;
  return g;
}

dpr_status check_camera(const dpr_camera* c) {
  if (!c) return fail(DPR_ERR_INVALID_ARGUMENT, "camera is NULL");
  if (c->width <= 0 || c->height <= 0 || (int64_t)c->width * c->height > (int64_t)1 << 30)
    return fail(DPR_ERR_INVALID_ARGUMENT, "camera size %dx%d invalid", c->width, c->height);
  if (!(c->fovy_deg > 0.0 && c->fovy_deg < 180.0))
    return fail(DPR_ERR_INVALID_ARGUMENT, "fovy_deg %g outside (0, 180)", c->fovy_deg);
  double f[3] = {c->center[0] - c->eye[0], c->center[1] - c->eye[1], c->center[2] - c->eye[2]};
  double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fn > 0.0) || !std::isfinite(fn)) return fail(DPR_ERR_INVALID_ARGUMENT, "camera eye == center");
  double r[3] = {f[1] * c->up[2] - f[2] * c->up[1], f[2] * c->up[0] - f[0] * c->up[2],
                 f[0] * c->up[1] - f[1] * c->up[0]};
  double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rn > 1e-12 * fn)) return fail(DPR_ERR_INVALID_ARGUMENT, "camera up is parallel to the view direction");
  return DPR_OK;
}

SceneG make_scene(const dpr_world_t* w) {
  SceneG s{};
  int64_t m = std::max(w->dims[0], std::max(w->dims[1], w->dims[2]));
  for (int a = 0; a < 3; ++a) s.dims[a] = (int)w->dims[a];
  s.h = 1.0 / (double)m;
  s.inv_h = (double)m;
  s.dt = (double)w->params.step_voxels * s.h;
  s.dt_f = (float)s.dt;
  s.density = w->density;
  s.ert = w->params.ert_threshold >= 1.f ? 2.f : w->params.ert_threshold;
  s.tf_lo = w->tf_lo;
  s.tf_scale = (float)(w->ntf - 1) / (w->tf_hi - w->tf_lo);
  s.ntf = w->ntf;
  if (w->iso_on) {
    s.iso_on = 1;
    s.iso = w->iso;
    s.iso_ka = w->iso_ka;
    s.iso_kd = w->iso_kd;
  }
  return s;
}

BrickG Brick::device_view(bool with_majorant, bool force_wide) const {
  BrickG g{};
  g.data = blocked;
  for (int a = 0; a < 3; ++a) {
    g.slo[a] = (int)(olo[a] - glo[a]);
    g.sdim[a] = sdim[a];
    g.olo[a] = (int)olo[a];
    g.ohi[a] = (int)ohi[a];
    g.mdim[a] = mdim[a];
  }
  g.bsy = (uint32_t)kBlockVoxels * (uint32_t)bdim[0];
  g.bsz = (uint32_t)kBlockVoxels * (uint32_t)bdim[0] * (uint32_t)bdim[1];
  g.majorant = with_majorant ? maj : nullptr;
  // an FP16 brick's addressing follows its layout (2-byte voxels: 64-bit offsets)
  if (dtype == DPR_F16)
    g.wide = half16 ? 1 : 0;
  else
    g.wide = force_wide || (uint64_t)bdim[0] * bdim[1] * bdim[2] * kBlockVoxels * 4u > 0xffffffffull;
  int sh = 0;
  while ((1 << sh) < mc) ++sh;
  g.mc_shift = sh;
  return g;
}

dpr_status ensure_majorants(dpr_world_t* w) {
  // bricks whose majorants predate the current TF, up to kMajJobs per launch
  MajJobs jobs{};
  jobs.iso_on = w->iso_on ? 1 : 0;
  jobs.iso = w->iso;
  Brick* pend[kMajJobs];
  auto flush = [&]() -> dpr_status {
    if (!jobs.n) return DPR_OK;
    DPR_HIP(launch_majorants(jobs, w->tf_dev, w->ntf, w->tf_lo, w->tf_hi, w->dev->stream));
    for (int j = 0; j < jobs.n; ++j) pend[j]->maj_tf_version = w->tf_version;
    jobs.n = 0;
    return DPR_OK;
  };
  for (auto& b : w->bricks) {
    if (b.maj_tf_version == w->tf_version) continue;
    jobs.ranges[jobs.n] = b.ranges;
    jobs.maj[jobs.n] = b.maj;
    jobs.count[jobs.n] = b.mdim[0] * b.mdim[1] * b.mdim[2];
    pend[jobs.n++] = &b;
    if (jobs.n == kMajJobs) {
      dpr_status st = flush();
      if (st != DPR_OK) return st;
    }
  }
  return flush();
}

// Composite tables are cached per (frames, ids) so repeated composites of the same
// frames (every dpr_render_frame) issue no host-to-device traffic at all.
dpr_status comp_table(dpr_device dev, const std::vector<const float4*>& rgba, const std::vector<const float*>& depth,
                      const std::vector<int32_t>& ids, CompTable** out, const std::vector<const int*>* counts,
                      const std::vector<int32_t>* caps) {
  const size_t k = rgba.size();
  std::vector<uint64_t> key;
  key.reserve(4 * k);
  for (size_t i = 0; i < k; ++i) {
    key.push_back((uint64_t)(uintptr_t)rgba[i]);
    key.push_back((uint64_t)(uintptr_t)depth[i]);
    key.push_back((uint64_t)(uint32_t)ids[i]);
    key.push_back(counts ? (uint64_t)(uintptr_t)(*counts)[i] : 0);
    key.push_back(caps ? (uint64_t)(uint32_t)(*caps)[i] : 0);
  }
  auto it = dev->comp_cache.find(key);
  if (it != dev->comp_cache.end()) {
    it->second.last_use = ++dev->use_clock;
    *out = it->second.dev;
    return DPR_OK;
  }
  if (dev->comp_cache.size() >= 64) {  // evict the least recently used table
    auto victim = dev->comp_cache.begin();
    for (auto j = dev->comp_cache.begin(); j != dev->comp_cache.end(); ++j)
      if (j->second.last_use < victim->second.last_use) victim = j;
    DPR_HIP(hipStreamSynchronize(dev->stream));
    dev_free(victim->second.dev);
    host_free(victim->second.host);
    dev->comp_cache.erase(victim);
  }
  CompEntry e;
  dpr_status hs = host_alloc((void**)&e.host, sizeof(CompTable), "composite table (host)");
  if (hs != DPR_OK) return hs;
  memset(e.host, 0, sizeof(CompTable));
  std::vector<int> order(k);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return ids[a] < ids[b]; });
  for (size_t r = 0; r < k; ++r) e.host->idrank[order[r]] = (int)r;
  for (size_t i = 0; i < k; ++i) {
    e.host->rgba[i] = rgba[i];
    e.host->depth[i] = depth[i];
    e.host->count[i] = counts ? (*counts)[i] : nullptr;
    e.host->cap[i] = caps ? (*caps)[i] : 0;
  }
  dpr_status st = dev_alloc((void**)&e.dev, sizeof(CompTable), "composite table");
  if (st != DPR_OK) {
    host_free(e.host);
    return st;
  }
  hipError_t he = hipMemcpyAsync(e.dev, e.host, sizeof(CompTable), hipMemcpyHostToDevice, dev->stream);
  if (he != hipSuccess) {
    dev_free(e.dev);
    host_free(e.host);
    return hip_fail(he, "hipMemcpyAsync(composite table)");
  }
  e.last_use = ++dev->use_clock;
  dev->comp_cache[key] = e;
  *out = e.dev;
  return DPR_OK;
}

dpr_status composite_frames(dpr_device dev, const dpr_frame* parts, const int32_t* ids, int32_t k, dpr_frame out) {
  if (!dev || !parts || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite: NULL argument");
  if (k < 1 || k > kMaxFrags) return fail(DPR_ERR_UNSUPPORTED, "dpr_composite: k=%d outside [1, %d]", k, kMaxFrags);
  std::vector<const float4*> rg(k);
  std::vector<const float*> dp(k);
  std::vector<int32_t> id(k);
  for (int i = 0; i < k; ++i) {
    const dpr_frame f = parts[i];
    if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite: part %d is NULL", i);
    if (f->dev != dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite: part %d belongs to another device", i);
    if (f->w != out->w || f->h != out->h)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite: part %d is %dx%d, out is %dx%d", i, f->w, f->h, out->w,
                  out->h);
    if (f->rgba == out->rgba || f->depth == out->depth)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite: out aliases part %d", i);
    rg[i] = (const float4*)f->rgba;
    dp[i] = f->depth;
    id[i] = ids ? ids[i] : i;
  }
  std::vector<int32_t> sorted = id;
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite: fragment ids must be distinct");
  CompTable* tab = nullptr;
  dpr_status st = comp_table(dev, rg, dp, id, &tab);
  if (st != DPR_OK) return st;
  const size_t P = (size_t)out->w * out->h;
  if (!dev->fix_count) {
    st = dev_alloc((void**)&dev->fix_count, 2 * sizeof(int), "composite fix-up counters");
    if (st != DPR_OK) return st;
    // zero once; the fix-up pass leaves both counters at zero after every call
    DPR_HIP(hipMemsetAsync(dev->fix_count, 0, 2 * sizeof(int), dev->stream));
  }
  if (!dev->comp_prior) {
    st = dev_alloc((void**)&dev->comp_prior, kCompPriorFloats * sizeof(float), "composite depth prior");
    if (st != DPR_OK) return st;
  }
  if (dev->fix_cap < P) {
    DPR_HIP(hipStreamSynchronize(dev->stream));
    dev_free(dev->fix_list);
    dev->fix_list = nullptr;
    dev->fix_cap = 0;
    st = dev_alloc((void**)&dev->fix_list, P * sizeof(int), "composite fix-up list");
    if (st != DPR_OK) return st;
    dev->fix_cap = P;
  }
  DPR_HIP(launch_composite(tab, k, (int)P, (float4*)out->rgba, out->depth, dev->fix_count, dev->fix_list,
                           dev->comp_prior, dev->cu_count, dev->stream));
  return DPR_OK;
}

}  // namespace dpr

using namespace dpr;

// ==================================================================== C ABI
extern "C" {

const char* dpr_last_error(void) { return g_last_error.c_str(); }
const char* dpr_version(void) { return "dpr 0.1 gfx950"; }

// ---------------------------------------------------------------- tile-shape cache
// {"version": 1, "entries": {"<key>": [w, h], ...}}; keys carry no quote or backslash.
static bool tune_cache_read(const char* path, std::map<std::string, std::pair<int, int>>& out) {
  out.clear();
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  std::string txt;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
  fclose(f);
  size_t i = txt.find("\"entries\"");
  if (i == std::string::npos) return false;
  i = txt.find('{', i);
  if (i == std::string::npos) return false;
  ++i;
  auto ws = [&]() {
    while (i < txt.size() && isspace((unsigned char)txt[i])) ++i;
  };
  auto integer = [&](int& v) {
    ws();
    size_t j = i;
    while (j < txt.size() && (isdigit((unsigned char)txt[j]) || (j == i && txt[j] == '-'))) ++j;
    if (j == i) return false;
    v = atoi(txt.substr(i, j - i).c_str());
    i = j;
    return true;
  };
  while (true) {
    ws();
    if (i >= txt.size()) return false;
    if (txt[i] == '}') return true;
    if (txt[i] == ',') {
      ++i;
      continue;
    }
    if (txt[i] != '"') return false;
    const size_t k1 = txt.find('"', i + 1);
    if (k1 == std::string::npos) return false;
    const std::string key = txt.substr(i + 1, k1 - i - 1);
    i = k1 + 1;
    ws();
    if (i >= txt.size() || txt[i] != ':') return false;
    ++i;
    ws();
    if (i >= txt.size() || txt[i] != '[') return false;
    ++i;
    int w = 0, h = 0;
    if (!integer(w)) return false;
    ws();
    if (i >= txt.size() || txt[i] != ',') return false;
    ++i;
    if (!integer(h)) return false;
    ws();
    if (i >= txt.size() || txt[i] != ']') return false;
    ++i;
    out[key] = {w, h};
  }
}

static bool tune_key_ok(const char* key) { return key && !strpbrk(key, "\"\\") && key[0]; }

dpr_status dpr_tune_cache_lookup(const char* path, const char* key, int32_t* found, int32_t* tw, int32_t* th) {
  if (!path || !found || !tw || !th || !tune_key_ok(key))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_tune_cache_lookup: NULL argument or a key with a quote");
  std::map<std::string, std::pair<int, int>> m;
  tune_cache_read(path, m);
  auto it = m.find(key);
  *found = it != m.end();
  if (*found) {
    *tw = it->second.first;
    *th = it->second.second;
  }
  return DPR_OK;
}

dpr_status dpr_tune_cache_store(const char* path, const char* key, int32_t tw, int32_t th) {
  if (!path || !tune_key_ok(key))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_tune_cache_store: NULL argument or a key with a quote");
  std::map<std::string, std::pair<int, int>> m;
  tune_cache_read(path, m);  // an unreadable file is replaced
  m[key] = {tw, th};
  std::string txt = "{\"version\": 1, \"entries\": {";
  bool first = true;
  for (const auto& e : m) {
    txt += first ? "\n  \"" : ",\n  \"";
    first = false;
    txt += e.first + "\": [" + std::to_string(e.second.first) + ", " + std::to_string(e.second.second) + "]";
  }
  txt += "\n}}\n";
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_tune_cache_store: cannot write %s", tmp.c_str());
  const bool ok = fwrite(txt.data(), 1, txt.size(), f) == txt.size();
  if (fclose(f) != 0 || !ok || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_tune_cache_store: cannot write %s", path);
  }
  return DPR_OK;
}

dpr_status dpr_alloc_stats(int64_t* allocations, int64_t* live) {
  if (allocations) *allocations = g_alloc_count.load();
  if (live) *live = g_alloc_live.load();
  return DPR_OK;
}

// ---------------------------------------------------------------- device
dpr_status dpr_device_create(int hip_device, void* hip_stream, dpr_device* out) {
  if (!out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_device_create: out is NULL");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0)
    return fail(DPR_ERR_DEVICE, "dpr_device_create: no HIP device visible (%s)",
                e != hipSuccess ? hipGetErrorString(e) : "count 0");
  if (hip_device < 0 || hip_device >= n)
    return fail(DPR_ERR_DEVICE, "dpr_device_create: device %d not in [0, %d)", hip_device, n);
  DPR_HIP(hipSetDevice(hip_device));
  hipDeviceProp_t prop;
  DPR_HIP(hipGetDeviceProperties(&prop, hip_device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DPR_ERR_UNSUPPORTED, "dpr_device_create: built for gfx950, device is %s", prop.gcnArchName);
  auto* d = new dpr_device_t;
  d->dev = hip_device;
  d->stream = (hipStream_t)hip_stream;
  d->cu_count = prop.multiProcessorCount;
  d->wave_size = prop.warpSize;
  const dpr_status st = noalloc_setup(d);
  if (st != DPR_OK) {
    delete d;
    return st;
  }
  *out = d;
  return DPR_OK;
}

dpr_status dpr_device_set_stream(dpr_device d, void* hip_stream) {
  if (!d) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_device_set_stream: NULL device");
  d->stream = (hipStream_t)hip_stream;
  return DPR_OK;
}

dpr_status dpr_device_sync(dpr_device d) {
  if (!d) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_device_sync: NULL device");
  DPR_HIP(hipStreamSynchronize(d->stream));
  DPR_HIP(hipGetLastError());
  return DPR_OK;
}

dpr_status dpr_device_info(dpr_device d, int32_t* cu, int32_t* ws) {
  if (!d) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_device_info: NULL device");
  if (cu) *cu = d->cu_count;
  if (ws) *ws = d->wave_size;
  return DPR_OK;
}

static void device_retain(dpr_device d) { ++d->refs; }

static void device_drop(dpr_device d) {
  if (--d->refs > 0) return;
  (void)hipStreamSynchronize(d->stream);
  for (auto& kv : d->comp_cache) {
    dev_free(kv.second.dev);
    host_free(kv.second.host);
  }
  dev_free(d->fix_count);
  dev_free(d->fix_list);
  dev_free(d->comp_prior);
  dev_free(d->tf_grad64);
  delete d;
}

void dpr_device_release(dpr_device d) {
  if (!d) return;
  device_drop(d);
}

// ---------------------------------------------------------------- world
dpr_status dpr_world_create(dpr_device d, const int64_t dims[3], dpr_world* out) {
  if (!d || !dims || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_create: NULL argument");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 2 || dims[a] > (1 << 20))
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_create: dims[%d]=%lld outside [2, 2^20]", a,
                  (long long)dims[a]);
  auto* w = new dpr_world_t;
  w->dev = d;
  device_retain(d);
  for (int a = 0; a < 3; ++a) w->dims[a] = dims[a];
  *out = w;
  return DPR_OK;
}

void dpr_world_release(dpr_world w) {
  if (!w) return;
  (void)hipStreamSynchronize(w->dev->stream);
  for (auto& b : w->bricks) {
    dev_free(b.linear);
    dev_free(b.blocked);
    dev_free(b.ranges);
    dev_free(b.maj);
  }
  for (auto f : w->partials) dpr_frame_release(f);
  if (w->batch) batch_state_free(w->batch);
  for (auto b : w->partial_batch)
    if (b) batch_state_free(b);
  if (w->path) path_state_free(w->path);
  dev_free(w->tf_dev);
  host_free(w->tf_host);
  if (w->tf_ev) (void)hipEventDestroy(w->tf_ev);
  dpr_device d = w->dev;
  delete w;
  device_drop(d);
}

dpr_status dpr_world_add_brick(dpr_world w, const void* voxels, dpr_dtype dtype, int on_device,
                               const int64_t lo[3], const int64_t hi[3], const int32_t glo[3], const int32_t ghi[3],
                               int32_t* brick_id) {
  if (!w || !voxels || !lo || !hi || !glo || !ghi || !brick_id)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_add_brick: NULL argument");
  if (dtype != DPR_F32 && dtype != DPR_F16)
    return fail(DPR_ERR_UNSUPPORTED, "dpr_world_add_brick: dtype %d is neither DPR_F32 nor DPR_F16", (int)dtype);
  Brick b{};
  uint64_t n = 1;
  for (int a = 0; a < 3; ++a) {
    if (!(0 <= lo[a] && lo[a] < hi[a] && hi[a] <= w->dims[a]))
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_add_brick: owned box axis %d [%lld, %lld) outside [0, %lld)",
                  a, (long long)lo[a], (long long)hi[a], (long long)w->dims[a]);
    if (glo[a] < 0 || ghi[a] < 0 || lo[a] - glo[a] < 0 || hi[a] + ghi[a] > w->dims[a])
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_add_brick: ghost layers on axis %d leave the domain", a);
    b.olo[a] = lo[a];
    b.ohi[a] = hi[a];
    b.glo[a] = glo[a];
    b.ghi[a] = ghi[a];
    b.sdim[a] = (int)(hi[a] - lo[a] + glo[a] + ghi[a]);
    if (b.sdim[a] < 2)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_add_brick: stored extent %d on axis %d < 2", b.sdim[a], a);
    b.bdim[a] = (b.sdim[a] + 7) / 8;
    n *= (uint64_t)b.sdim[a];
  }
  uint64_t blocked = (uint64_t)b.bdim[0] * b.bdim[1] * b.bdim[2] * kBlockVoxels;
  if (blocked > 0xFFFFFFFFull)
    return fail(DPR_ERR_UNSUPPORTED, "dpr_world_add_brick: brick of %llu blocked voxels exceeds 2^32",
                (unsigned long long)blocked);
  b.dtype = dtype;
  size_t bytes = n * b.elem();
  dpr_status st = dev_alloc(&b.linear, bytes + kLinearSlack, "brick voxels");
  if (st != DPR_OK) return st;
  hipError_t e = hipMemcpyAsync(b.linear, voxels, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                w->dev->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(w->dev->stream);
  if (e != hipSuccess) {
    dev_free(b.linear);
    return hip_fail(e, "dpr_world_add_brick: copy");
  }
  w->bricks.push_back(b);
  w->committed = false;
  ++w->geo_version;
  *brick_id = (int32_t)w->bricks.size() - 1;
  return DPR_OK;
}

// Host-only partition check (no device call): disjoint owned boxes, ghost layers on
// every owned face interior to the domain, optional tiling (DPR_REQUIRE_TILING=1).
static dpr_status check_partition_arrays(const int64_t dims[3], int32_t n, const int64_t* lo, const int64_t* hi,
                                         const int32_t* glo, const int32_t* ghi) {
  if (n <= 0) return fail(DPR_ERR_INVALID_STATE, "partition: no bricks");
  for (int32_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      const int64_t l = lo[3 * i + a], h = hi[3 * i + a];
      if (!(0 <= l && l < h && h <= dims[a]))
        return fail(DPR_ERR_INVALID_ARGUMENT, "partition: brick %d axis %d owned [%lld, %lld) outside [0, %lld)", i,
                    a, (long long)l, (long long)h, (long long)dims[a]);
      if (glo[3 * i + a] < 0 || ghi[3 * i + a] < 0 || l - glo[3 * i + a] < 0 || h + ghi[3 * i + a] > dims[a])
        return fail(DPR_ERR_INVALID_ARGUMENT, "partition: brick %d ghost layers on axis %d leave the domain", i, a);
      if (l > 0 && glo[3 * i + a] < 1)
        return fail(DPR_ERR_INVALID_ARGUMENT,
                    "partition: brick %d has no ghost layer on its interior low face of axis %d", i, a);
      if (h < dims[a] && ghi[3 * i + a] < 1)
        return fail(DPR_ERR_INVALID_ARGUMENT,
                    "partition: brick %d has no ghost layer on its interior high face of axis %d", i, a);
    }
    for (int32_t j = i + 1; j < n; ++j) {
      bool overlap = true;
      for (int a = 0; a < 3; ++a) overlap &= lo[3 * i + a] < hi[3 * j + a] && lo[3 * j + a] < hi[3 * i + a];
      if (overlap) return fail(DPR_ERR_INVALID_ARGUMENT, "partition: owned boxes of bricks %d and %d overlap", i, j);
    }
  }
  const char* t = getenv("DPR_REQUIRE_TILING");
  if (t && t[0] == '1') {
    long double vol = 0;
    for (int32_t i = 0; i < n; ++i)
      vol += (long double)(hi[3 * i] - lo[3 * i]) * (hi[3 * i + 1] - lo[3 * i + 1]) * (hi[3 * i + 2] - lo[3 * i + 2]);
    if (vol != (long double)dims[0] * dims[1] * dims[2])
      return fail(DPR_ERR_INVALID_ARGUMENT, "partition: bricks do not tile the global domain");
  }
  return DPR_OK;
}

static dpr_status check_partition(const dpr_world_t* w) {
  const auto& B = w->bricks;
  if (B.empty()) return fail(DPR_ERR_INVALID_STATE, "dpr_world_commit: world has no bricks");
  std::vector<int64_t> lo, hi;
  std::vector<int32_t> glo, ghi;
  for (const auto& b : B)
    for (int a = 0; a < 3; ++a) {
      lo.push_back(b.olo[a]);
      hi.push_back(b.ohi[a]);
      glo.push_back(b.glo[a]);
      ghi.push_back(b.ghi[a]);
    }
  return check_partition_arrays(w->dims, (int32_t)B.size(), lo.data(), hi.data(), glo.data(), ghi.data());
}

dpr_status dpr_check_partition(const int64_t dims[3], int32_t n, const int64_t* lo, const int64_t* hi,
                               const int32_t* glo, const int32_t* ghi) {
  if (!dims || !lo || !hi || !glo || !ghi) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_check_partition: NULL argument");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 2) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_check_partition: dims[%d] < 2", a);
  return check_partition_arrays(dims, n, lo, hi, glo, ghi);
}

dpr_status dpr_check_camera(const dpr_camera* c) { return check_camera(c); }

dpr_status dpr_world_commit(dpr_world w) {
  if (!w) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_commit: NULL world");
  dpr_status st = check_partition(w);
  if (st != DPR_OK) return st;
  for (const auto& b : w->bricks)
    if (!b.linear) {
      if (w->committed) return DPR_OK;  // nothing to rebuild
      return fail(DPR_ERR_INVALID_STATE,
                  "dpr_world_commit: the linear copies were released and the bricks, the macrocell edge or the FP16 "
                  "layout flags changed since the last commit");
    }
  const int mc = w->params.macrocell_cells;
  // FP16 layout, one for the whole world (the batched kernel reads every brick the
  // same way): 2-byte voxels when asked for (or 64-bit offsets were), or when some
  // brick's voxel-pair copy would reach 4 GiB; else voxel pairs
  bool f16_halves = (w->params.flags & (DPR_FLAG_F16_HALVES | DPR_FLAG_WIDE_OFFSETS)) != 0;
  for (const auto& b : w->bricks)
    f16_halves |= b.dtype == DPR_F16 &&
                  (uint64_t)b.bdim[0] * b.bdim[1] * b.bdim[2] * kBlockVoxels * 4u >= kF16HalvesFrom;
  for (auto& b : w->bricks) {
    // a change of layout re-allocates the blocked copy
    const bool half16 = b.dtype == DPR_F16 && f16_halves;
    if (b.blocked && half16 != b.half16) {
      DPR_HIP(hipStreamSynchronize(w->dev->stream));
      dev_free(b.blocked);
      b.blocked = nullptr;
    }
    b.half16 = half16;
    if (!b.blocked) {
      size_t bytes = (size_t)b.bdim[0] * b.bdim[1] * b.bdim[2] * kBlockVoxels * b.blocked_elem() + kPairSlack;
      st = dev_alloc(&b.blocked, bytes, "blocked brick");
      if (st != DPR_OK) return st;
      // padding voxels (beyond the stored dims) are never written by the commit
      DPR_HIP(hipMemsetAsync(b.blocked, 0, bytes, w->dev->stream));
    }
    int md[3];
    for (int a = 0; a < 3; ++a) md[a] = (int)((b.ohi[a] - b.olo[a] + mc - 1) / mc);
    if (!b.ranges || b.mc != mc || md[0] != b.mdim[0] || md[1] != b.mdim[1] || md[2] != b.mdim[2]) {
      dev_free(b.ranges);
      dev_free(b.maj);
      b.ranges = nullptr;
      b.maj = nullptr;
      size_t cnt = (size_t)md[0] * md[1] * md[2];
      // the ranges, then the commit's two partial ranges per macrocell (the
      // x-windows that straddle two commit waves' column spans)
      st = dev_alloc((void**)&b.ranges, 3 * cnt * sizeof(float2), "macrocell ranges");
      if (st != DPR_OK) return st;
      st = dev_alloc((void**)&b.maj, cnt * sizeof(float), "macrocell majorants");
      if (st != DPR_OK) return st;
    }
    for (int a = 0; a < 3; ++a) b.mdim[a] = md[a];
    b.mc = mc;
    b.maj_tf_version = 0;
  }
  std::vector<McBrick> mcb;
  for (auto& b : w->bricks)
    mcb.push_back({b.linear, b.device_view(false), b.ranges, b.ranges + (size_t)b.mdim[0] * b.mdim[1] * b.mdim[2],
                   b.dtype == DPR_F16, b.half16});
  DPR_HIP(launch_commit(mcb.data(), (int)mcb.size(), mc, w->dev->cu_count, w->dev->stream));
  // (stream-ordered: later renders on the device stream see the new data; the
  // host does not wait)
  w->committed = true;
  ++w->commit_version;
  return DPR_OK;
}

dpr_status dpr_world_release_linear(dpr_world w) {
  if (!w) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_release_linear: NULL world");
  if (!w->committed) return fail(DPR_ERR_INVALID_STATE, "dpr_world_release_linear: world not committed");
  DPR_HIP(hipStreamSynchronize(w->dev->stream));  // the commit reads them
  for (auto& b : w->bricks) {
    dev_free(b.linear);
    b.linear = nullptr;
  }
  return DPR_OK;
}

dpr_status dpr_world_brick_count(dpr_world w, int32_t* n) {
  if (!w || !n) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_brick_count: NULL argument");
  *n = (int32_t)w->bricks.size();
  return DPR_OK;
}

dpr_status dpr_world_brick_macrocells(dpr_world w, int32_t id, int32_t md[3], float* ranges, float* maj,
                                      size_t capacity) {
  if (!w || !md) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_brick_macrocells: NULL argument");
  if (!w->committed) return fail(DPR_ERR_INVALID_STATE, "dpr_world_brick_macrocells: world not committed");
  if (id < 0 || id >= (int)w->bricks.size())
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_brick_macrocells: brick %d does not exist", id);
  Brick& b = w->bricks[id];
  size_t cnt = (size_t)b.mdim[0] * b.mdim[1] * b.mdim[2];
  if ((ranges || maj) && capacity < cnt)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_brick_macrocells: capacity %zu < %zu", capacity, cnt);
  if (maj) {
    if (!w->tf_set) return fail(DPR_ERR_INVALID_STATE, "dpr_world_brick_macrocells: no transfer function set");
    dpr_status st = ensure_majorants(w);
    if (st != DPR_OK) return st;
  }
  DPR_HIP(hipStreamSynchronize(w->dev->stream));
  if (ranges) DPR_HIP(hipMemcpy(ranges, b.ranges, cnt * sizeof(float2), hipMemcpyDeviceToHost));
  if (maj) DPR_HIP(hipMemcpy(maj, b.maj, cnt * sizeof(float), hipMemcpyDeviceToHost));
  for (int a = 0; a < 3; ++a) md[a] = b.mdim[a];
  return DPR_OK;
}

dpr_status dpr_world_brick_blocked(dpr_world w, int32_t id, int32_t bdim[3], int32_t* elem_bytes, void* host,
                                   size_t capacity) {
  if (!w || !bdim || !elem_bytes) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_brick_blocked: NULL argument");
  if (!w->committed) return fail(DPR_ERR_INVALID_STATE, "dpr_world_brick_blocked: world not committed");
  if (id < 0 || id >= (int)w->bricks.size())
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_brick_blocked: brick %d does not exist", id);
  const Brick& b = w->bricks[id];
  const size_t bytes = (size_t)b.bdim[0] * b.bdim[1] * b.bdim[2] * kBlockVoxels * b.blocked_elem();
  for (int a = 0; a < 3; ++a) bdim[a] = b.bdim[a];
  *elem_bytes = (int32_t)b.blocked_elem();
  if (!host) return DPR_OK;
  if (capacity < bytes)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_world_brick_blocked: capacity %zu < %zu bytes", capacity, bytes);
  DPR_HIP(hipStreamSynchronize(w->dev->stream));
  DPR_HIP(hipMemcpy(host, b.blocked, bytes, hipMemcpyDeviceToHost));
  return DPR_OK;
}

dpr_status dpr_set_transfer_function(dpr_world w, const float* rgba, int32_t n, float lo, float hi, float density) {
  if (!w || !rgba) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_transfer_function: NULL argument");
  if (n < 2 || n > kMaxTF) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_transfer_function: n_entries %d", n);
  if (!(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_transfer_function: value range [%g, %g]", lo, hi);
  if (!(density >= 0.f) || !std::isfinite(density))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_transfer_function: density %g", density);
  for (int i = 0; i < 4 * n; ++i)
    if (!(rgba[i] >= 0.f) || !std::isfinite(rgba[i]))
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_transfer_function: entry %d is negative or not finite", i / 4);
  if (w->ntf != n) {
    dev_free(w->tf_dev);
    w->tf_dev = nullptr;
    w->ntf = 0;
    dpr_status st = dev_alloc((void**)&w->tf_dev, (size_t)n * sizeof(float4), "transfer function");
    if (st != DPR_OK) return st;
    w->ntf = n;
  }
  // stage through pinned host memory so the upload is stream-ordered and the host
  // does not wait for the device; the staging buffer is reused once the previous
  // upload has been consumed
  if (!w->tf_host) {
    dpr_status hs = host_alloc((void**)&w->tf_host, kMaxTF * sizeof(float4), "transfer function staging");
    if (hs != DPR_OK) return hs;
    DPR_HIP(hipEventCreateWithFlags(&w->tf_ev, hipEventDisableTiming));
  }
  if (w->tf_ev_pending) DPR_HIP(hipEventSynchronize(w->tf_ev));
  memcpy(w->tf_host, rgba, (size_t)n * sizeof(float4));
  DPR_HIP(hipMemcpyAsync(w->tf_dev, w->tf_host, (size_t)n * sizeof(float4), hipMemcpyHostToDevice, w->dev->stream));
  DPR_HIP(hipEventRecord(w->tf_ev, w->dev->stream));
  w->tf_ev_pending = true;
  w->tf_lo = lo;
  w->tf_hi = hi;
  w->density = density;
  w->tf_set = true;
  ++w->tf_version;
  return DPR_OK;
}

dpr_status dpr_set_isosurface(dpr_world w, int32_t enable, float value, float ambient, float diffuse) {
  if (!w) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_isosurface: NULL world");
  if (enable) {
    if (!std::isfinite(value)) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_isosurface: value %g", value);
    if (!(ambient >= 0.f) || !std::isfinite(ambient) || !(diffuse >= 0.f) || !std::isfinite(diffuse))
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_isosurface: ambient %g, diffuse %g", ambient, diffuse);
    w->iso = value;
    w->iso_ka = ambient;
    w->iso_kd = diffuse;
  }
  w->iso_on = enable != 0;
  ++w->tf_version;  // the majorants carry the skip classes of the surface
  return DPR_OK;
}

dpr_status dpr_set_camera(dpr_world w, const dpr_camera* c) {
  if (!w) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_camera: NULL world");
  dpr_status st = check_camera(c);
  if (st != DPR_OK) return st;
  w->cam = *c;
  w->cam_set = true;
  return DPR_OK;
}

dpr_status dpr_set_render_params(dpr_world w, const dpr_render_params* p) {
  if (!w || !p) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_render_params: NULL argument");
  if (!(p->step_voxels > 0.f && p->step_voxels <= 1.f))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_render_params: step_voxels %g outside (0, 1]", p->step_voxels);
  if (!(p->ert_threshold > 0.f) || std::isnan(p->ert_threshold))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_render_params: ert_threshold %g", p->ert_threshold);
  int mc = p->macrocell_cells;
  if (mc < 2 || mc > 64 || (mc & (mc - 1)))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_set_render_params: macrocell_cells %d not a power of two in [2, 64]",
                mc);
  if (mc != w->params.macrocell_cells) w->committed = false;
  // the FP16 layout (and with it the FP16 addressing) is chosen at commit
  if ((p->flags ^ w->params.flags) & (DPR_FLAG_F16_HALVES | DPR_FLAG_WIDE_OFFSETS)) w->committed = false;
  w->params = *p;
  return DPR_OK;
}

// ---------------------------------------------------------------- frames
dpr_status dpr_frame_create(dpr_device d, int32_t wd, int32_t ht, dpr_frame* out) {
  if (!d || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_create: NULL argument");
  if (wd <= 0 || ht <= 0 || (int64_t)wd * ht > (int64_t)1 << 30)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_create: size %dx%d", wd, ht);
  auto* f = new dpr_frame_t;
  f->dev = d;
  f->w = wd;
  f->h = ht;
  f->owned = true;
  size_t px = (size_t)wd * ht;
  dpr_status st = dev_alloc((void**)&f->rgba, px * 16, "frame rgba");
  if (st == DPR_OK) st = dev_alloc((void**)&f->depth, px * 4, "frame depth");
  if (st != DPR_OK) {
    dev_free(f->rgba);
    delete f;
    return st;
  }
  device_retain(d);
  *out = f;
  return DPR_OK;
}

dpr_status dpr_frame_wrap(dpr_device d, int32_t wd, int32_t ht, float* rgba, float* depth, dpr_frame* out) {
  if (!d || !out || !rgba || !depth) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_wrap: NULL argument");
  if (wd <= 0 || ht <= 0 || (int64_t)wd * ht > (int64_t)1 << 30)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_wrap: size %dx%d", wd, ht);
  if (((uintptr_t)rgba & 15) || ((uintptr_t)depth & 3))
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_wrap: rgba must be 16-byte and depth 4-byte aligned");
  auto* f = new dpr_frame_t;
  f->dev = d;
  f->w = wd;
  f->h = ht;
  f->rgba = rgba;
  f->depth = depth;
  f->owned = false;
  device_retain(d);
  *out = f;
  return DPR_OK;
}

dpr_status dpr_frame_attach_counts(dpr_frame f, int32_t* counts) {
  if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_attach_counts: NULL frame");
  f->counts = counts;
  return DPR_OK;
}

dpr_status dpr_frame_map(dpr_frame f, const float** rgba, const float** depth) {
  if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_map: NULL frame");
  DPR_HIP(hipStreamSynchronize(f->dev->stream));
  DPR_HIP(hipGetLastError());
  if (rgba) *rgba = f->rgba;
  if (depth) *depth = f->depth;
  return DPR_OK;
}

dpr_status dpr_frame_unmap(dpr_frame f) {
  if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_unmap: NULL frame");
  return DPR_OK;
}

dpr_status dpr_frame_read(dpr_frame f, float* rgba, float* depth) {
  if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_frame_read: NULL frame");
  DPR_HIP(hipStreamSynchronize(f->dev->stream));
  size_t px = (size_t)f->w * f->h;
  if (rgba) DPR_HIP(hipMemcpy(rgba, f->rgba, px * 16, hipMemcpyDeviceToHost));
  if (depth) DPR_HIP(hipMemcpy(depth, f->depth, px * 4, hipMemcpyDeviceToHost));
  return DPR_OK;
}

void dpr_frame_release(dpr_frame f) {
  if (!f) return;
  if (f->owned) {
    (void)hipStreamSynchronize(f->dev->stream);
    dev_free(f->rgba);
    dev_free(f->depth);
  }
  dpr_device d = f->dev;
  delete f;
  device_drop(d);
}

// ---------------------------------------------------------------- render / composite
static dpr_status check_renderable(dpr_world w, const char* who) {
  if (!w->committed) return fail(DPR_ERR_INVALID_STATE, "%s: world not committed", who);
  if (!w->tf_set) return fail(DPR_ERR_INVALID_STATE, "%s: no transfer function set", who);
  if (!w->cam_set) return fail(DPR_ERR_INVALID_STATE, "%s: no camera set", who);
  return DPR_OK;
}

static dpr_status render_brick(dpr_world w, int id, dpr_frame out) {
  const Brick& b = w->bricks[id];
  const bool skip = !(w->params.flags & DPR_FLAG_NO_SKIP);
  SceneG sc = make_scene(w);
  CamG cam = make_cam(w->cam);
  const BrickG g = b.device_view(skip, w->params.flags & DPR_FLAG_WIDE_OFFSETS);
  DPR_HIP(launch_march(sc, g, cam, w->tf_dev, b.dtype == DPR_F16, skip, (float4*)out->rgba,
                       out->depth, out->counts, w->dev->stream));
  return DPR_OK;
}

dpr_status dpr_render_partial(dpr_world w, int32_t id, dpr_frame out) {
  if (!w || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_partial: NULL argument");
  dpr_status st = check_renderable(w, "dpr_render_partial");
  if (st != DPR_OK) return st;
  if (id < 0 || id >= (int)w->bricks.size())
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_partial: brick %d does not exist", id);
  if (out->w != w->cam.width || out->h != w->cam.height)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_partial: frame %dx%d != camera %dx%d", out->w, out->h,
                w->cam.width, w->cam.height);
  if (out->dev != w->dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_partial: frame of another device");
  st = ensure_majorants(w);
  if (st != DPR_OK) return st;
  // the persistent kernel, unless the plain launch is asked for or per-pixel
  // sample counts are (only the plain launch writes them)
  if (!(w->params.flags & DPR_FLAG_PLAIN) && !out->counts) return render_partial_batched(w, id, out);
  return render_brick(w, id, out);
}

dpr_status dpr_measure_gather(dpr_world w, int32_t id, const int32_t* counts, float* sink) {
  if (!w || !counts || !sink) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_measure_gather: NULL argument");
  dpr_status st = check_renderable(w, "dpr_measure_gather");
  if (st != DPR_OK) return st;
  if (id < 0 || id >= (int)w->bricks.size())
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_measure_gather: brick %d does not exist", id);
  st = ensure_majorants(w);
  if (st != DPR_OK) return st;
  const Brick& b = w->bricks[id];
  const bool skip = !(w->params.flags & DPR_FLAG_NO_SKIP);
  DPR_HIP(launch_gather_probe(make_scene(w), b.device_view(skip, w->params.flags & DPR_FLAG_WIDE_OFFSETS),
                              make_cam(w->cam), b.dtype == DPR_F16, counts, sink, w->dev->stream));
  return DPR_OK;
}

dpr_status dpr_composite(dpr_device d, const dpr_frame* parts, const int32_t* ids, int32_t k, dpr_frame out) {
  return composite_frames(d, parts, ids, k, out);
}

// ---------------------------------------------------------------- deep frames
static dpr_status deep_frame_checks(dpr_device d, int32_t wd, int32_t ht, int32_t cap, const char* who) {
  if (!d) return fail(DPR_ERR_INVALID_ARGUMENT, "%s: NULL device", who);
  if (wd <= 0 || ht <= 0 || (int64_t)wd * ht > (int64_t)1 << 30)
    return fail(DPR_ERR_INVALID_ARGUMENT, "%s: size %dx%d", who, wd, ht);
  if (cap < 1 || cap > 255) return fail(DPR_ERR_INVALID_ARGUMENT, "%s: capacity %d outside [1, 255]", who, cap);
  return DPR_OK;
}

dpr_status dpr_deep_frame_create(dpr_device d, int32_t wd, int32_t ht, int32_t cap, dpr_deep_frame* out) {
  if (!out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_deep_frame_create: NULL out");
  dpr_status st = deep_frame_checks(d, wd, ht, cap, "dpr_deep_frame_create");
  if (st != DPR_OK) return st;
  auto* f = new dpr_deep_frame_t;
  f->dev = d;
  device_retain(d);  // dropped by dpr_deep_frame_release, also on the failure path below
  f->w = wd;
  f->h = ht;
  f->cap = cap;
  f->owned = true;
  const size_t px = (size_t)wd * ht, lay = px * cap;
  if ((st = dev_alloc((void**)&f->counts, px * sizeof(int), "deep frame counts")) != DPR_OK ||
      (st = dev_alloc((void**)&f->rgba, lay * sizeof(float4), "deep frame rgba")) != DPR_OK ||
      (st = dev_alloc((void**)&f->depth, lay * sizeof(float), "deep frame depth")) != DPR_OK ||
      (st = dev_alloc((void**)&f->ids, lay * sizeof(int), "deep frame ids")) != DPR_OK) {
    dpr_deep_frame_release(f);
    return st;
  }
  *out = f;
  return DPR_OK;
}

dpr_status dpr_deep_frame_wrap(dpr_device d, int32_t wd, int32_t ht, int32_t cap, int32_t* counts, float* rgba,
                               float* depth, int32_t* ids, dpr_deep_frame* out) {
  if (!out || !counts || !rgba || !depth || !ids)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_deep_frame_wrap: NULL argument");
  dpr_status st = deep_frame_checks(d, wd, ht, cap, "dpr_deep_frame_wrap");
  if (st != DPR_OK) return st;
  auto* f = new dpr_deep_frame_t;
  f->dev = d;
  f->w = wd;
  f->h = ht;
  f->cap = cap;
  f->counts = counts;
  f->rgba = (float4*)rgba;
  f->depth = depth;
  f->ids = ids;
  device_retain(d);
  *out = f;
  return DPR_OK;
}

void dpr_deep_frame_release(dpr_deep_frame f) {
  if (!f) return;
  if (f->owned) {
    (void)hipStreamSynchronize(f->dev->stream);
    dev_free(f->counts);
    dev_free(f->rgba);
    dev_free(f->depth);
    dev_free(f->ids);
  }
  dpr_device d = f->dev;
  delete f;
  device_drop(d);
}

dpr_status dpr_composite_deep(dpr_device dev, const dpr_deep_frame* parts, int32_t k, dpr_frame out) {
  if (!dev || !parts || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_deep: NULL argument");
  if (k < 1) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_deep: k = %d", k);
  if (out->dev != dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_deep: out belongs to another device");
  if (k > kMaxFrags) return fail(DPR_ERR_UNSUPPORTED, "dpr_composite_deep: %d parts > %d", k, kMaxFrags);
  std::vector<const float4*> rg;
  std::vector<const float*> dp;
  std::vector<int32_t> ranks;
  std::vector<const int*> cnt;
  std::vector<int32_t> caps;
  for (int j = 0; j < k; ++j) {
    const dpr_deep_frame f = parts[j];
    if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_deep: part %d is NULL", j);
    if (f->dev != dev)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_deep: part %d belongs to another device", j);
    if (f->w != out->w || f->h != out->h)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_deep: part %d is %dx%d, out is %dx%d", j, f->w, f->h,
                  out->w, out->h);
    if (f->rank < 0)
      return fail(DPR_ERR_INVALID_STATE, "dpr_composite_deep: part %d was not rendered by dpr_render_deep", j);
    rg.push_back(f->rgba);
    dp.push_back(f->depth);
    ranks.push_back(f->rank);
    cnt.push_back(f->counts);
    caps.push_back(f->cap);
  }
  // Ties in depth order as the fragments' ids: inside a part the layers are in
  // (depth, id) order, and ids of different parts differ in their rank, so the
  // kernel ranks fragments by (depth, part rank, layer)
  std::vector<int32_t> sr = ranks;
  std::sort(sr.begin(), sr.end());
  if (std::adjacent_find(sr.begin(), sr.end()) != sr.end())
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_deep: the parts must come from distinct ranks");
  CompTable* tab = nullptr;
  dpr_status st = comp_table(dev, rg, dp, ranks, &tab, &cnt, &caps);
  if (st != DPR_OK) return st;
  DPR_HIP(launch_composite_deep(tab, k, (int)((size_t)out->w * out->h), (float4*)out->rgba, out->depth,
                                dev->stream));
  return DPR_OK;
}

dpr_status dpr_render_frame(dpr_world w, dpr_frame out) {
  if (!w || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_frame: NULL argument");
  dpr_status st = check_renderable(w, "dpr_render_frame");
  if (st != DPR_OK) return st;
  if (out->w != w->cam.width || out->h != w->cam.height)
    return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_frame: frame %dx%d != camera %dx%d", out->w, out->h,
                w->cam.width, w->cam.height);
  const int K = (int)w->bricks.size();
  if (K > kMaxFrags) return fail(DPR_ERR_UNSUPPORTED, "dpr_render_frame: %d bricks > %d", K, kMaxFrags);
  if (out->dev != w->dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_render_frame: frame of another device");
  bool mixed = false;
  for (const auto& b : w->bricks) mixed |= b.dtype != w->bricks[0].dtype;
  if (!(w->params.flags & DPR_FLAG_PLAIN) && !mixed) {
    st = ensure_majorants(w);
    if (st != DPR_OK) return st;
    return render_frame_batched(w, out);
  }
  bool resize = (int)w->partials.size() != K;
  for (auto f : w->partials) resize |= f->w != out->w || f->h != out->h;
  if (resize) {
    for (auto f : w->partials) dpr_frame_release(f);
    w->partials.clear();
    for (int i = 0; i < K; ++i) {
      dpr_frame f = nullptr;
      st = dpr_frame_create(w->dev, out->w, out->h, &f);
      if (st != DPR_OK) return st;
      w->partials.push_back(f);
    }
  }
  st = ensure_majorants(w);
  if (st != DPR_OK) return st;
  for (int i = 0; i < K; ++i) {
    st = render_brick(w, i, w->partials[i]);
    if (st != DPR_OK) return st;
  }
  std::vector<int32_t> ids(K);
  std::iota(ids.begin(), ids.end(), 0);
  return composite_frames(w->dev, w->partials.data(), ids.data(), K, out);
}

}  // extern "C"
