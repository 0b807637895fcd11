// Index spans of the streaming commit, shared by the commit kernel and its host
// launcher (and checked on the host by the test suite).
#pragma once

#include <algorithm>

#include <hip/hip_runtime.h>

namespace dpr {

constexpr int kCmCols = 128;  // stored x-voxels of a commit wave's span (16 lanes x 8)

// Window, write core and loaded range of macrocells [m0, m1) along one axis of n
// stored voxels whose first owned voxel is stored at g (align: 2 for the row
// pairs of y and z; the kernel takes y one macrocell at a time and derives its z
// stages from it).  Macrocell m covers owned voxels [mc m - 1, mc m + mc], clipped
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

// x: wave k takes the stored columns [kCmCols k, kCmCols (k + 1)) (whole cache
// lines, shared with no other wave).  The macrocells whose x-window meets that
// span are [m0, m1] (none when m0 > m1).  A window (at most mc + 2 <= 66 columns)
// meets one or two spans: the span holding its first column computes the range
// over its part of the window as partial 0, the other span (if any) as partial
// 1; a span that holds the whole window writes an empty partial 1.
struct XCells {
  int m0, m1;
};
__host__ __device__ inline XCells xspan_cells(int k, int md, int mc, int g, int n) {
  const int x0 = kCmCols * k, x1 = std::min(n - 1, x0 + kCmCols - 1);
  XCells c;
  // first m whose window ends at or after x0 (window end mc m + mc + g, clipped to n - 1 >= x0)
  c.m0 = x0 - mc - g <= 0 ? 0 : (x0 - mc - g + mc - 1) / mc;
  // last m whose window starts at or before x1 (start mc m - 1 + g; macrocell 0's: max(0, g - 1))
  c.m1 = x1 + 1 - g < 0 ? -1 : std::min(md - 1, (x1 + 1 - g) / mc);
  return c;
}

// Row pairs (even first row zp: rows zp, zp + 1) that stage s of a z-segment of
// macrocells [m0, m1) visits, as even zp in [lo, hi):
//  - s = m0 - 1, the prelude: pairs before the segment's first core that hold
//    rows of macrocell m0's window (read only; their writer is the segment below);
//  - s in [m0, m1): pairs whose even row lies in macrocell s's core (written);
//  - s = m1, the postlude: pairs after the last core that hold rows of macrocell
//    m1 - 1's window (read only).
// A row visited in stage s lies in the windows of macrocells s - 1, s, s + 1 only,
// and macrocell s - 1's window is complete once stage s is done.
struct ZStage {
  int lo, hi;
  bool own;
};
__host__ __device__ inline ZStage z_stage(int s, int m0, int m1, int md, int mc, int g, int n) {
  ZStage st{0, 0, false};
  if (s < m0) {
    if (m0 > 0) {
      const AxisSpan a = axis_span(m0, m0 + 1, md, mc, g, n, 2);
      st.lo = a.ws & ~1;
      st.hi = a.cs;
    }
  } else if (s >= m1) {
    if (m1 < md) {
      const AxisSpan a = axis_span(m1 - 1, m1, md, mc, g, n, 2);
      st.lo = (a.ce + 1) & ~1;
      st.hi = a.we + 1;
    }
  } else {
    const AxisSpan a = axis_span(s, s + 1, md, mc, g, n, 2);
    st.lo = (a.cs + 1) & ~1;
    st.hi = a.ce;
    st.own = true;
  }
  st.hi = std::max(st.lo, st.hi);
  return st;
}

}  // namespace dpr
