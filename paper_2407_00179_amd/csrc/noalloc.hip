// Allocation-free sort-last composite (dpr_composite_noalloc).
//
// The same kernels as dpr_composite, with every piece of device scratch they use
// -- the fragment table, the sampled depth prior, the fix-up counters and the
// fix-up pixel list -- carved out of one fixed array of this library instead of
// memory allocated on first use.  Each GPU the library runs on holds its own copy
// of the array until the process ends; its device address is looked up once per
// device when the first device handle for that GPU is created.  The table is
// written by a small kernel whose arguments carry it, so a call issues no
// allocation and no host-to-device copy.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "runtime.hpp"

namespace dpr {

namespace {

constexpr size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

constexpr size_t kNaTableOff = 0;
constexpr size_t kNaPriorOff = kNaTableOff + align256(sizeof(CompTable));
constexpr size_t kNaCountOff = kNaPriorOff + align256(kCompPriorFloats * sizeof(float));
constexpr size_t kNaListOff = kNaCountOff + 256;
constexpr size_t kNaBytes = kNaListOff + kNoAllocMaxPixels * sizeof(int);

}  // namespace

// Only the device address looked up below may be passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
void* g_na_ptr[kNaMaxDevices] = {};

// Table entries k0 .. k0 + n - 1 (n <= kNaChunk) travel in the kernel arguments.
constexpr int kNaChunk = 32;
struct TableChunk {
  const float4* rgba[kNaChunk];
  const float* depth[kNaChunk];
  int idrank[kNaChunk];
  int k0, n;
};

__global__ __launch_bounds__(64) void table_fill_kernel(TableChunk c, CompTable* tab, int* fix_count) {
  const int i = threadIdx.x;
  if (i < c.n) {
    tab->rgba[c.k0 + i] = c.rgba[i];
    tab->depth[c.k0 + i] = c.depth[i];
    tab->idrank[c.k0 + i] = c.idrank[i];
    tab->count[c.k0 + i] = nullptr;
    tab->cap[c.k0 + i] = 0;
  }
  // the fix-up counters must start at zero (the fix-up pass also leaves them so)
  if (c.k0 == 0 && i < 2) fix_count[i] = 0;
}

}  // namespace

dpr_status noalloc_setup(dpr_device d) {
  void* p = nullptr;
  if (d->dev >= 0 && d->dev < kNaMaxDevices) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    p = g_na_ptr[d->dev];
    if (!p) {
      // d->dev is the current device (set by dpr_device_create)
      DPR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      g_na_ptr[d->dev] = p;
    }
  } else {
    DPR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  }
  d->noalloc_scratch = p;
  return DPR_OK;
}

}  // namespace dpr

using namespace dpr;

extern "C" dpr_status dpr_composite_noalloc(dpr_device dev, const dpr_frame* parts, const int32_t* ids, int32_t k,
                                            dpr_frame out) {
  if (!dev || !parts || !out) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_noalloc: NULL argument");
  if (k < 1 || k > kMaxFrags)
    return fail(DPR_ERR_UNSUPPORTED, "dpr_composite_noalloc: k=%d outside [1, %d]", k, kMaxFrags);
  if (out->dev != dev) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_noalloc: out belongs to another device");
  const size_t P = (size_t)out->w * out->h;
  if (P > kNoAllocMaxPixels)
    return fail(DPR_ERR_UNSUPPORTED, "dpr_composite_noalloc: %zu pixels exceed the allocation-free maximum of %zu",
                P, kNoAllocMaxPixels);
  if (!dev->noalloc_scratch) return fail(DPR_ERR_INVALID_STATE, "dpr_composite_noalloc: no scratch on this device");
  // every table entry on the stack: nothing is allocated, on the host either
  TableChunk chunk[kMaxFrags / kNaChunk];
  for (int i = 0; i < k; ++i) {
    const dpr_frame f = parts[i];
    if (!f) return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_noalloc: part %d is NULL", i);
    if (f->dev != dev)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_noalloc: part %d belongs to another device", i);
    if (f->w != out->w || f->h != out->h)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_noalloc: part %d is %dx%d, out is %dx%d", i, f->w, f->h,
                  out->w, out->h);
    if (f->rgba == out->rgba || f->depth == out->depth)
      return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_noalloc: out aliases part %d", i);
    // the rank of this part's id among the k ids breaks depth ties
    const int32_t id = ids ? ids[i] : i;
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const int32_t o = ids ? ids[j] : j;
      if (j != i && o == id)
        return fail(DPR_ERR_INVALID_ARGUMENT, "dpr_composite_noalloc: fragment ids must be distinct");
      rank += o < id;
    }
    TableChunk& c = chunk[i / kNaChunk];
    c.rgba[i % kNaChunk] = (const float4*)f->rgba;
    c.depth[i % kNaChunk] = f->depth;
    c.idrank[i % kNaChunk] = rank;
  }
  unsigned char* base = (unsigned char*)dev->noalloc_scratch;
  CompTable* tab = (CompTable*)(base + kNaTableOff);
  float* prior = (float*)(base + kNaPriorOff);
  int* fix_count = (int*)(base + kNaCountOff);
  int* fix_list = (int*)(base + kNaListOff);
  for (int c0 = 0; c0 < k; c0 += kNaChunk) {
    TableChunk& c = chunk[c0 / kNaChunk];
    c.k0 = c0;
    c.n = std::min(kNaChunk, k - c0);
    hipLaunchKernelGGL(table_fill_kernel, dim3(1), dim3(64), 0, dev->stream, c, tab, fix_count);
  }
  DPR_HIP(launch_composite(tab, k, (int)P, (float4*)out->rgba, out->depth, fix_count, fix_list, prior, dev->cu_count,
                           dev->stream));
  return DPR_OK;
}
