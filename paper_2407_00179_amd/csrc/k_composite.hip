// Sort-last compositor over K whole frames (dpr_composite).
//
// Fast path: a workgroup of 4 waves walks a run of 256-pixel strips, each wave
// taking one 64-pixel tile of every strip, so the four waves read neighbouring
// bytes of every source.  Per tile the wave ranks the sources by (key, id rank)
// -- the tile order -- where a source's key is its nearest depth over the last
// tile of the run in which it had fragments (a sampled nearest depth over the
// whole frame before that).  It then walks the sources in tile order, reading each
// lane's depth (coalesced) and RGBA only for live fragments, and composites front
// to back on the fly while checking, per pixel, that its live fragments really
// arrive in (depth, id) order.  Every depth and every live RGBA is read once.
// Neighbouring pixels almost always share one order (convex bricks: a separating
// plane orders two bricks identically for every ray; per-rank depth slabs), so
// nothing is stored per pixel and no LDS staging limits occupancy.  A pixel whose
// fragments break the tile order is recomposited in exact (depth, id) order with
// the same arithmetic, so it gets the same bits, through a fix-up list that a
// second pass works off with the fully general per-wave sort (composite_wave).
//
// Few sources (K <= 16): one pixel per lane, whose K keys are sorted in registers
// by a fixed compare-exchange network and composited with the same arithmetic, so
// again the same bits; no prior pass, no tile order, no fix-up list.
#include <algorithm>

#include "composite.h"
#include "device_common.h"
#include "kernels.h"

namespace dpr {

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}

// Sampled nearest depth of every source over about kPriorTiles 64-pixel tiles
// spread evenly over the frame (an odd tile stride, so the samples also spread
// over the columns).  Block (s, k) reduces its slice of the samples of source k
// into prior[k * kPriorSlices + s].
constexpr int kPriorSlices = 4;
constexpr int kPriorTiles = 512;

__device__ __forceinline__ int prior_stride(int n_tiles) { return (n_tiles / kPriorTiles) | 1; }

__global__ __launch_bounds__(256) void composite_prior_kernel(const CompTable* __restrict__ tab, int P,
                                                              float* __restrict__ prior) {
  __shared__ float wmin[4];
  const int k = blockIdx.y, slice = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float* __restrict__ d = tab->depth[k];
  const int n_tiles = (P + 63) / 64;
  const int stride = prior_stride(n_tiles);
  const int n_samp = (n_tiles + stride - 1) / stride;
  constexpr int step = kPriorSlices * 4;
  float m = INFINITY;
  for (int j0 = slice + kPriorSlices * wave; j0 < n_samp; j0 += step * 8) {
    float z[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * step;
      const int p = j * stride * 64 + lane;
      z[u] = (j < n_samp && p < P) ? d[p] : INFINITY;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fminf(m, z[u]);
  }
  m = wave_min(m);
  if (lane == 0) wmin[wave] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    prior[k * kPriorSlices + slice] = fminf(fminf(wmin[0], wmin[1]), fminf(wmin[2], wmin[3]));
}

// Minimum over the 64 lanes with DPP row shifts and row broadcasts (VALU only);
// the result is wave-uniform.
#define DPR_DPP_MIN(v, ctrl, row_mask)                                                                        \
  v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), ctrl, row_mask, \
                                                          0xf, false)))
__device__ __forceinline__ float wave_min_dpp(float v) {
  DPR_DPP_MIN(v, 0x111, 0xf);  // row_shr:1
  DPR_DPP_MIN(v, 0x112, 0xf);  // row_shr:2
  DPR_DPP_MIN(v, 0x114, 0xf);  // row_shr:4
  DPR_DPP_MIN(v, 0x118, 0xf);  // row_shr:8 -> lane 15 of each row holds the row minimum
  DPR_DPP_MIN(v, 0x142, 0xa);  // row_bcast:15 into rows 1 and 3
  DPR_DPP_MIN(v, 0x143, 0xc);  // row_bcast:31 into rows 2 and 3 -> lane 63 holds the minimum
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
#undef DPR_DPP_MIN

template <int KMAX, int B, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void composite_fast_kernel(const CompTable* __restrict__ tab, int K, int P,
                                                             const float* __restrict__ prior,
                                                             float4* __restrict__ out_rgba,
                                                             float* __restrict__ out_depth, int* __restrict__ fix_count,
                                                             int* __restrict__ fix_list, int strips_per_group) {
  __shared__ const float4* prgba[KMAX];
  __shared__ const float* pdepth[KMAX];
  __shared__ int prank[KMAX];
  __shared__ float key0[KMAX];
  __shared__ float rep[4][KMAX];
  __shared__ unsigned char order[4][KMAX];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = threadIdx.x; k < K; k += 256) {
    prgba[k] = tab->rgba[k];
    pdepth[k] = tab->depth[k];
    prank[k] = tab->idrank[k];
    float m = prior[k * kPriorSlices];
#pragma unroll
    for (int s = 1; s < kPriorSlices; ++s) m = fminf(m, prior[k * kPriorSlices + s]);
    key0[k] = m;
  }
  __syncthreads();
  // the workgroup walks a run of 256-pixel strips, wave w taking the w-th 64-pixel
  // tile of each strip, so the four waves read neighbouring bytes of every source
  const int n_tiles = (P + 63) / 64;
  const int n_strips = (n_tiles + 3) / 4;
  const int s0 = blockIdx.x * strips_per_group;
  const int s1 = min(n_strips, s0 + strips_per_group);
  const int t0 = s0 * 4 + wave;
  if (s0 >= s1 || t0 >= n_tiles) return;  // (no block-wide barrier follows)
  // keys for the first tile: nearest depths over that tile, the sampled nearest
  // depth for sources absent from it
  {
    const int p = t0 * 64 + lane;
    for (int k0 = 0; k0 < K; k0 += B) {
      float z[B];
#pragma unroll
      for (int u = 0; u < B; ++u) z[u] = (p < P && k0 + u < K) ? pdepth[k0 + u][p] : INFINITY;
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const float m = wave_min_dpp(z[u]);
        if (lane == 0 && k0 + u < K) rep[wave][k0 + u] = m < INFINITY ? m : key0[k0 + u];
      }
    }
  }
  for (int t = t0; t < min(n_tiles, s1 * 4); t += 4) {
    // tile order by (key, id rank); a source's key is its nearest depth over the
    // last tile of the run where it had fragments (this tile, for the first one);
    // any order gives the same bits, a good one just keeps pixels on the fast path
    // (the previous tile's order is kept when the new keys leave it sorted)
    bool sorted = t != t0;
    if (sorted) {
      for (int i = lane; i + 1 < K; i += 64) {
        const int a = order[wave][i], b = order[wave][i + 1];
        const float ka = rep[wave][a], kb = rep[wave][b];
        sorted &= (ka < kb) || (ka == kb && prank[a] < prank[b]);
      }
      sorted = __all(sorted);
    }
    if (!sorted) {
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // reads of the old order done before it is rewritten
      for (int k = lane; k < K; k += 64) {
        const float rk = rep[wave][k];
        const int ik = prank[k];
        int r = 0;
        for (int j = 0; j < K; ++j) {
          const float rj = rep[wave][j];
          r += (rj < rk) || (rj == rk && prank[j] < ik);
        }
        order[wave][r] = (unsigned char)k;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // LDS writes visible to the whole wave
    }
    const int p = t * 64 + lane;
    const bool live_px = p < P;
    float tr = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, ca = 0.f, zfirst = INFINITY;
    float lz = -INFINITY;
    int lr = -1;
    bool bad = !live_px;
    // sources in batches of B: source indices and depths of a batch, then RGBA of
    // its live fragments; the next batch's depths are requested before this batch
    // is composited, so one memory round trip per batch is exposed
    int ku[B];
    float zu[B];
    auto fetch = [&](int i1, int* kk, float* zz) {
#pragma unroll
      for (int u = 0; u < B; ++u) {
        kk[u] = (i1 + u < K) ? order[wave][i1 + u] : 0;
        zz[u] = (live_px && i1 + u < K) ? pdepth[kk[u]][p] : INFINITY;
      }
    };
    fetch(0, ku, zu);
    for (int i0 = 0; i0 < K; i0 += B) {
      float4 f[B];
#pragma unroll
      for (int u = 0; u < B; ++u)
        f[u] = (zu[u] < INFINITY && !bad) ? prgba[ku[u]][p] : make_float4(0.f, 0.f, 0.f, 0.f);
      int kn[B];
      float zn[B];
      fetch(i0 + B, kn, zn);
#pragma unroll
      for (int u = 0; u < B; ++u) {
        // nearest depth of this source over the tile, the key for the next tiles
        const float m = wave_min_dpp(zu[u]);
        if (lane == 0 && i0 + u < K && m < INFINITY) rep[wave][ku[u]] = m;
        if (zu[u] < INFINITY && !bad) {
          const int r = prank[ku[u]];
          if (zu[u] > lz || (zu[u] == lz && r > lr)) {
            if (lr < 0) zfirst = zu[u];
            cr = fmaf(tr, f[u].x, cr);
            cg = fmaf(tr, f[u].y, cg);
            cb = fmaf(tr, f[u].z, cb);
            ca = fmaf(tr, f[u].w, ca);
            tr *= 1.f - f[u].w;
            lz = zu[u];
            lr = r;
          } else {
            bad = true;  // out of tile order: the general sort takes this pixel
          }
        }
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        ku[u] = kn[u];
        zu[u] = zn[u];
      }
    }
    if (live_px) {
      if (bad) {
        const int slot = atomicAdd(fix_count, 1);
        fix_list[slot] = p;
      } else {
        out_rgba[p] = make_float4(cr, cg, cb, ca);
        out_depth[p] = zfirst;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// General path for the pixels of the fix-up list: one wave per 64 listed pixels,
// persistent over the list (its length is read on the device).  The last
// workgroup to finish clears the list length and the finish count, so the
// counters are zero again for the next call without a separate clear.
template <int KMAX>
__global__ __launch_bounds__(64) void composite_fixup_kernel(const CompTable* __restrict__ tab, int K,
                                                             float4* __restrict__ out_rgba,
                                                             float* __restrict__ out_depth,
                                                             int* __restrict__ fix_count,
                                                             const int* __restrict__ fix_list) {
  __shared__ CompLDS<KMAX> s;
  __shared__ const float4* prgba[KMAX];
  __shared__ const float* pdepth[KMAX];
  const int lane = threadIdx.x;
  const int n = *fix_count;
  if (blockIdx.x * 64 < n) {
    for (int k = lane; k < K; k += 64) {
      prgba[k] = tab->rgba[k];
      pdepth[k] = tab->depth[k];
    }
    __syncthreads();
  }
  for (int base = blockIdx.x * 64; base < n; base += gridDim.x * 64) {
    const bool live = base + lane < n;
    const int p = live ? fix_list[base + lane] : 0;
    float4 c;
    float z;
    composite_wave<KMAX>(
        s, K, live, [&](int k) { return pdepth[k][p]; }, [&](int k) { return prgba[k][p]; },
        [&](int k) { return tab->idrank[k]; }, c, z);
    if (live) {
      out_rgba[p] = c;
      out_depth[p] = z;
    }
    __syncthreads();
  }
  if (lane == 0) {
    __threadfence();
    if (atomicAdd(fix_count + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(fix_count, 0);
      atomicExch(fix_count + 1, 0);
    }
  }
}

// Few sources: lane = pixel.  Keys (depth, id rank), with a fragment that is not
// live (depth not below +inf, NaN included) keyed +inf, are sorted by Batcher's
// odd-even merge network over KS slots (padding slots: +inf); the network's
// indices are compile-time constants once unrolled, so the keys stay in
// registers.  The id rank and the source index travel as one word (rank << 8 |
// source; ranks and sources are below 256).  The live fragments' RGBA are then
// requested 4 at a time in sorted order and composited front to back.  Each lane
// walks pixels with a grid stride and requests the next pixel's depths before
// this pixel's RGBA.
template <int KS>
__global__ __launch_bounds__(256) void composite_small_kernel(const CompTable* __restrict__ tab, int K, int P,
                                                              float4* __restrict__ out_rgba,
                                                              float* __restrict__ out_depth) {
  // RGBA pointers are picked per lane after the sort, so they sit in LDS; the
  // depth pointers are wave-uniform and read from the table into scalar registers
  __shared__ const float4* prgba[KS];
  __shared__ uint32_t prk[KS];
  for (int k = threadIdx.x; k < KS; k += blockDim.x) {
    prgba[k] = k < K ? tab->rgba[k] : nullptr;
    prk[k] = ((k < K ? (uint32_t)tab->idrank[k] : 0xffffffu) << 8) | (uint32_t)k;
  }
  __syncthreads();
  const int stride = gridDim.x * blockDim.x;
  auto load_depths = [&](int pp, float* z) {
#pragma unroll
    for (int u = 0; u < KS; ++u) z[u] = (u < K && pp < P) ? ld_global(tab->depth[u], pp) : INFINITY;
  };
  float zc[KS];
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  load_depths(p, zc);
  for (; p < P; p += stride) {
    float zn[KS];
    load_depths(p + stride, zn);
    float z[KS];
    uint32_t rk[KS];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      z[u] = zc[u] < INFINITY ? zc[u] : INFINITY;
      rk[u] = prk[u];
    }
#pragma unroll
    for (int q = 1; q < KS; q <<= 1) {
#pragma unroll
      for (int d = q; d >= 1; d >>= 1) {
#pragma unroll
        for (int j = d % q; j + d < KS; j += 2 * d) {
#pragma unroll
          for (int i = 0; i < d && i + j + d < KS; ++i) {
            const int a = i + j, b = i + j + d;
            if ((a / (2 * q)) == (b / (2 * q))) {
              const bool sw = z[b] < z[a] || (z[b] == z[a] && rk[b] < rk[a]);
              const float za = z[a], zb = z[b];
              const uint32_t ra = rk[a], rb = rk[b];
              z[a] = sw ? zb : za;
              z[b] = sw ? za : zb;
              rk[a] = sw ? rb : ra;
              rk[b] = sw ? ra : rb;
            }
          }
        }
      }
    }
    float tr = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, ca = 0.f;
#pragma unroll
    for (int b0 = 0; b0 < KS; b0 += 4) {
      if (!(z[b0] < INFINITY)) break;  // sorted: no live fragment from here on
      float4 f[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        f[u] = z[b0 + u] < INFINITY ? prgba[rk[b0 + u] & 0xffu][p] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (z[b0 + u] < INFINITY) {
          cr = fmaf(tr, f[u].x, cr);
          cg = fmaf(tr, f[u].y, cg);
          cb = fmaf(tr, f[u].z, cb);
          ca = fmaf(tr, f[u].w, ca);
          tr *= 1.f - f[u].w;
        }
      }
    }
    out_rgba[p] = make_float4(cr, cg, cb, ca);
    out_depth[p] = z[0];
#pragma unroll
    for (int u = 0; u < KS; ++u) zc[u] = zn[u];
  }
}

// Resident waves per SIMD of the fast kernel: the register budget that keeps
// every workgroup of the persistent grid resident at once.
constexpr int kFastWavesPerSimd = 5;

template <int KMAX>
static void launch_k(const CompTable* tab, int k, int n_pixels, float4* out_rgba, float* out_depth, int* fix_count,
                     int* fix_list, float* prior, int cu_count, hipStream_t st) {
  if (n_pixels <= 0) return;
  hipLaunchKernelGGL(composite_prior_kernel, dim3(kPriorSlices, k), dim3(256), 0, st, tab, n_pixels, prior);
  // workgroups of 4 waves walk runs of 256-pixel strips, one resident grid
  // (kFastWavesPerSimd workgroups per CU)
  const int n_strips = (n_pixels + 255) / 256;
  const int groups = cu_count * kFastWavesPerSimd;
  const int per = (n_strips + groups - 1) / groups;
  const int blocks = (n_strips + per - 1) / per;
  hipLaunchKernelGGL((composite_fast_kernel<KMAX, 8, kFastWavesPerSimd>), dim3(blocks), dim3(256), 0, st, tab, k,
                     n_pixels, prior, out_rgba, out_depth, fix_count, fix_list, per);
  hipLaunchKernelGGL(composite_fixup_kernel<KMAX>, dim3(cu_count), dim3(64), 0, st, tab, k, out_rgba, out_depth,
                     fix_count, fix_list);
}

// Merge of deep frames (dpr_composite_deep).  Table entry r describes part r:
// rgba[r] / depth[r] are its layer-major arrays (layer l of pixel p at l * P + p),
// count[r] its per-pixel fragment counts, idrank[r] its place in rank order.
// One thread per pixel.  A fragment's key is (depth, part rank, layer); the thread
// takes the pixel's fragments in passes, each keeping the kSel nearest keys beyond
// the last one composited -- in registers, sorted by a branch-free insertion --
// and compositing them front to back with the same "over" as composite_wave, so a
// pixel with n live fragments costs ceil(n / kSel) passes over its depths.  The
// parts' layers need not be sorted for this: every live fragment is ranked.
constexpr int kSel = 8;

__device__ __forceinline__ bool key_less(float za, int ka, float zb, int kb) {
  return za < zb || (za == zb && ka < kb);
}

__global__ __launch_bounds__(256) void deep_merge_kernel(const CompTable* __restrict__ tab, int R, int P,
                                                         float4* __restrict__ out_rgba,
                                                         float* __restrict__ out_depth) {
  __shared__ const float* pdepth[kMaxFrags];
  __shared__ const int* pcount[kMaxFrags];
  __shared__ int pcap[kMaxFrags];
  __shared__ int pkey[kMaxFrags];                  // rank-order index << 8
  __shared__ const float4* rgba_by_rank[kMaxFrags];
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    const int q = tab->idrank[r];
    pdepth[r] = tab->depth[r];
    pcount[r] = tab->count[r];
    pcap[r] = tab->cap[r];
    pkey[r] = q << 8;
    rgba_by_rank[q] = tab->rgba[r];
  }
  __syncthreads();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const size_t sP = (size_t)P;
  float lz = -INFINITY;  // last key composited
  int lk = -1;
  float tr = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, ca = 0.f, znear = INFINITY;
  int done = 0, n = 0;
  do {
    float z[kSel];
    int kk[kSel];
#pragma unroll
    for (int j = 0; j < kSel; ++j) {
      z[j] = INFINITY;
      kk[j] = 0;
    }
    int m = 0;
    n = 0;
    for (int r0 = 0; r0 < R; r0 += 8) {
      int c[8];
#pragma unroll
      // a count is trusted only up to the part's capacity (layers beyond it do not
      // exist), and a fragment whose depth is not below +inf (NaN included) is not
      // live, as in the flat compositor
      for (int u = 0; u < 8; ++u) c[u] = r0 + u < R ? min(max(pcount[r0 + u][p], 0), pcap[r0 + u]) : 0;
      // every part's first layer is requested at once; deeper layers (rare) in the loop
      float d0[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) d0[u] = c[u] > 0 ? pdepth[r0 + u][p] : INFINITY;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (c[u] <= 0) continue;
        const float* dz = pdepth[r0 + u] + p;
        const int kb = pkey[r0 + u];
        for (int l = 0; l < c[u]; ++l) {
          const float d = l == 0 ? d0[u] : dz[(size_t)l * sP];
          if (!(d < INFINITY)) continue;
          ++n;
          const int key = kb | l;
          if (!key_less(lz, lk, d, key)) continue;                             // composited already
          if (m == kSel && !key_less(d, key, z[kSel - 1], kk[kSel - 1])) continue;  // beyond this pass
          int pos = 0;
#pragma unroll
          for (int j = 0; j < kSel; ++j) pos += (j < m) && key_less(z[j], kk[j], d, key);
#pragma unroll
          for (int j = kSel - 1; j > 0; --j) {
            z[j] = j > pos ? z[j - 1] : (j == pos ? d : z[j]);
            kk[j] = j > pos ? kk[j - 1] : (j == pos ? key : kk[j]);
          }
          if (pos == 0) {
            z[0] = d;
            kk[0] = key;
          }
          m = m < kSel ? m + 1 : kSel;
        }
      }
    }
    if (m == 0) break;  // nothing left beyond the last key (every pass selects at least one otherwise)
    if (done == 0) znear = z[0];
#pragma unroll
    for (int j = 0; j < kSel; ++j) {
      if (j < m) {
        const float4 f = rgba_by_rank[kk[j] >> 8][(size_t)(kk[j] & 255) * sP + p];
        cr = fmaf(tr, f.x, cr);
        cg = fmaf(tr, f.y, cg);
        cb = fmaf(tr, f.z, cb);
        ca = fmaf(tr, f.w, ca);
        tr *= 1.f - f.w;
        lz = z[j];
        lk = kk[j];
      }
    }
    done += m;
  } while (done < n);
  out_rgba[p] = make_float4(cr, cg, cb, ca);
  out_depth[p] = znear;
}

hipError_t launch_composite_deep(const CompTable* table_dev, int parts, int n_pixels, float4* out_rgba,
                                 float* out_depth, hipStream_t st) {
  if (n_pixels <= 0) return hipSuccess;
  hipLaunchKernelGGL(deep_merge_kernel, dim3((n_pixels + 255) / 256), dim3(256), 0, st, table_dev, parts, n_pixels,
                     out_rgba, out_depth);
  return hipGetLastError();
}

template <int KS>
static void launch_small(const CompTable* tab, int k, int n_pixels, float4* out_rgba, float* out_depth, int cu_count,
                         hipStream_t st) {
  if (n_pixels <= 0) return;
  // one resident grid (the workgroups a CU holds at once, as the runtime reports
  // for this kernel), each lane walking a few pixels with a grid stride
  static const int per_cu = [] {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, composite_small_kernel<KS>, 256, 0) != hipSuccess) {
      (void)hipGetLastError();  // a guess of 4 is fine; keep the failed query out of the launch's status
      b = 4;
    }
    return std::max(1, b);
  }();
  const int blocks = (int)std::min<long long>(((long long)n_pixels + 255) / 256, (long long)cu_count * per_cu);
  hipLaunchKernelGGL(composite_small_kernel<KS>, dim3(blocks), dim3(256), 0, st, tab, k, n_pixels, out_rgba,
                     out_depth);
}

hipError_t launch_composite(const CompTable* table_dev, int k, int n_pixels, float4* out_rgba, float* out_depth,
                            int* fix_count, int* fix_list, float* prior, int cu_count, hipStream_t st) {
  if (k <= 8)
    launch_small<8>(table_dev, k, n_pixels, out_rgba, out_depth, cu_count, st);
  else if (k <= 16)
    launch_small<16>(table_dev, k, n_pixels, out_rgba, out_depth, cu_count, st);
  else if (k <= 64)
    launch_k<64>(table_dev, k, n_pixels, out_rgba, out_depth, fix_count, fix_list, prior, cu_count, st);
  else if (k <= 128)
    launch_k<128>(table_dev, k, n_pixels, out_rgba, out_depth, fix_count, fix_list, prior, cu_count, st);
  else
    launch_k<256>(table_dev, k, n_pixels, out_rgba, out_depth, fix_count, fix_list, prior, cu_count, st);
  return hipGetLastError();
}

}  // namespace dpr
