// Index spans of the one-pass commit along one axis, shared by the commit kernel
// and its host launcher (and checked on the host by the test suite).
#pragma once

#include <algorithm>

#include <hip/hip_runtime.h>

namespace dpr {

constexpr int kCmCols = 384;  // x-voxels a commit workgroup may load (3 chunks of 128)

// Window, write core and loaded range of macrocells [m0, m1) along one axis of n
// stored voxels whose first owned voxel is stored at g (align: 4 for x-runs, 2
// for row pairs).  Macrocell m covers owned voxels [mc m - 1, mc m + mc], clipped
// to the stored range; the cores of consecutive spans partition [0, n) (the first
// extended down to 0, the last up to n); the loaded range covers the window and
// every aligned group whose first voxel lies in the core.
struct AxisSpan {
  int ws, we;  // window, inclusive
  int cs, ce;  // write core, exclusive end
  int ls, le;  // loaded, inclusive; ls a multiple of align
};
__host__ __device__ inline AxisSpan axis_span(int m0, int m1, int md, int mc, int g, int n, int align) {
  AxisSpan a;
  a.ws = std::max(0, mc * m0 - 1 + g);
  a.we = std::min(n - 1, mc * m1 + g);
  a.cs = m0 == 0 ? 0 : mc * m0 + g;
  a.ce = m1 == md ? n : mc * m1 + g;
  a.ls = std::min(a.ws, a.cs) & ~(align - 1);
  a.le = std::min(n - 1, std::max(a.we, a.ce - 1) | (align - 1));
  return a;
}

// Macrocells per workgroup along x (sx stored voxels, first owned at g, md
// macrocells): the most whose loaded x-range fits kCmCols.
inline int commit_per_chunk(int sx, int g, int md, int mc) {
  for (int pc = std::min(md, kCmCols / mc); pc > 1; --pc) {
    bool fits = true;
    for (int m0 = 0; m0 < md && fits; m0 += pc) {
      const AxisSpan a = axis_span(m0, std::min(md, m0 + pc), md, mc, g, sx, 4);
      fits = a.le - a.ls + 1 <= kCmCols;
    }
    if (fits) return pc;
  }
  return 1;
}

}  // namespace dpr
