// Per-wave sort-last compositing of 64 pixels, shared by dpr_composite's kernel
// and the batched renderer's tile compositor so both produce the same bits.
//
// One wave owns 64 pixels.  All K depths of those pixels are staged in LDS with
// coalesced loads (4 B per fragment, the only bytes read for empty fragments).
// The wave first orders the K fragment sources by their nearest depth in the
// tile; neighbouring pixels almost always share that order (convex bricks, depth
// slabs), so each lane's insertion sort over its live fragments is nearly an
// append-only pass.  RGBA is then fetched only for live fragments, in sorted
// order, which keeps lanes on the same source and the 16 B loads coalesced.
// Sort key: (depth, id rank); "over" on all four premultiplied channels:
// C += T rgba_i, T *= 1 - alpha_i.
#pragma once

#include "device_common.h"

namespace dpr {

template <int KMAX>
struct CompLDS {
  float zs[KMAX][65];
  unsigned char lst[KMAX][64];
  float rep[KMAX];
  int rank[KMAX];
  unsigned char order[KMAX];
};

// Steps 1-3 of the per-wave compositor: stage the depths, order the sources for
// the tile, and leave each lane's live fragments sorted by (depth, id rank) in
// s.lst[0 .. n-1][lane]; returns n.
// depth_of(k): depth of source k at this lane's pixel (only called for live lanes);
// rank_of(k): id rank of source k (distinct per source).
template <int KMAX, typename DepthF, typename RankF>
__device__ __forceinline__ int sort_wave(CompLDS<KMAX>& s, int K, bool live_px, DepthF depth_of, RankF rank_of) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < K; k += 64) {
    s.rank[k] = rank_of(k);
    s.order[k] = (unsigned char)k;  // every slot holds a valid source even if ranks collided
  }
  // 1. depths of the tile, coalesced per source.  Large K runs at a few waves per
  //    CU (LDS-bound), so each lane keeps up to 64 loads in flight in registers.
  constexpr int B = KMAX < 64 ? KMAX : 64;
  for (int k0 = 0; k0 < K; k0 += B) {
    float v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = (live_px && k0 + u < K) ? depth_of(k0 + u) : INFINITY;
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (k0 + u < K) s.zs[k0 + u][lane] = v[u];
  }
  __syncthreads();
  // 2. tile order of the sources by (nearest depth in the tile, id rank)
  for (int k = lane; k < K; k += 64) {
    float m = INFINITY;
    for (int i = 0; i < 64; ++i) m = fminf(m, s.zs[k][i]);
    s.rep[k] = m;
  }
  __syncthreads();
  for (int k = lane; k < K; k += 64) {
    const float rk = s.rep[k];
    const int ik = s.rank[k];
    int r = 0;
    for (int j = 0; j < K; ++j) {
      const float rj = s.rep[j];
      r += (rj < rk) || (rj == rk && s.rank[j] < ik);
    }
    s.order[r] = (unsigned char)k;
  }
  __syncthreads();
  // 3. per-lane sorted list of live fragments (insertion sort, nearly append-only)
  int n = 0;
  float lz = -INFINITY;
  int lr = -1;
  for (int i = 0; i < K; ++i) {
    const int k = s.order[i];
    const float z = s.zs[k][lane];
    if (!(z < INFINITY)) continue;
    const int r = s.rank[k];
    if (z > lz || (z == lz && r > lr)) {
      s.lst[n][lane] = (unsigned char)k;
      lz = z;
      lr = r;
    } else {
      int pos = n;
      while (pos > 0) {
        const int kk = s.lst[pos - 1][lane];
        const float zz = s.zs[kk][lane];
        if (zz < z || (zz == z && s.rank[kk] < r)) break;
        s.lst[pos][lane] = (unsigned char)kk;
        --pos;
      }
      s.lst[pos][lane] = (unsigned char)k;
    }
    ++n;
  }
  return n;
}

// depth_of(k): depth of source k at this lane's pixel (only called for live lanes);
// rgba_of(k): its RGBA; rank_of(k): id rank of source k (distinct per source).
template <int KMAX, typename DepthF, typename RgbaF, typename RankF>
__device__ __forceinline__ void composite_wave(CompLDS<KMAX>& s, int K, bool live_px, DepthF depth_of,
                                               RgbaF rgba_of, RankF rank_of, float4& out, float& out_z) {
  const int lane = threadIdx.x & 63;
  const int n = sort_wave<KMAX>(s, K, live_px, depth_of, rank_of);
  // 4. front-to-back over, RGBA fetched for live fragments only, up to F loads in
  //    flight per lane (a partial batch is predicated, not walked one load at a time)
  float tr = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, ca = 0.f;
  constexpr int F = KMAX <= 16 ? 8 : 16;
  for (int i = 0; i < n; i += F) {
    float4 f[F];
#pragma unroll
    for (int u = 0; u < F; ++u) f[u] = i + u < n ? rgba_of(s.lst[i + u][lane]) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < F; ++u) {
      if (i + u < n) {
        cr = fmaf(tr, f[u].x, cr);
        cg = fmaf(tr, f[u].y, cg);
        cb = fmaf(tr, f[u].z, cb);
        ca = fmaf(tr, f[u].w, ca);
        tr *= 1.f - f[u].w;
      }
    }
  }
  out = make_float4(cr, cg, cb, ca);
  out_z = n ? s.zs[s.lst[0][lane]][lane] : INFINITY;
}

}  // namespace dpr
