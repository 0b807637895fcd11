// Host check of the streaming commit's index spans (commit_span.h): for brick
// extents, ghost widths and macrocell edges drawn at random,
//  - x, in aligned spans of kCmCols columns: every macrocell's window
//    [mc m - 1, mc m + mc] (owned coordinates, clipped) is the union of its parts
//    in the spans that list it, partial 0 is written by exactly one span (the one
//    holding the window's first column) and partial 1 by exactly one;
//  - y, one macrocell per span, in row pairs: every stored row is written by
//    exactly one span, which loads it, loaded ranges stay inside the stored range
//    and start aligned, and every window lies inside the loaded range of its span;
//  - z, streamed in segments of macrocells: every row pair is written by exactly
//    one stage of one segment, every row of a macrocell's window is visited by
//    its segment no later than the stage that completes it, and a row visited in
//    stage s lies only in the windows of macrocells s - 1, s, s + 1.
// The 3-D ownership of the kernel is the product of the three axes' ownerships.
#include <cstdio>
#include <random>
#include <vector>

#include "commit_span.h"

using dpr::AxisSpan;

static int fails = 0;
#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      if (++fails < 20) {                  \
        std::printf("FAIL %s: ", #c);      \
        std::printf(__VA_ARGS__);          \
        std::printf("\n");                 \
      }                                    \
    }                                      \
  } while (0)

static void check_axis(int own, int glo, int ghi, int mc, int align, int per) {
  const int n = own + glo + ghi, md = (own + mc - 1) / mc;
  std::vector<int> writers(n, 0), loaded_by_writer(n, 0);
  for (int m0 = 0; m0 < md; m0 += per) {
    const int m1 = std::min(md, m0 + per);
    const AxisSpan a = dpr::axis_span(m0, m1, md, mc, glo, n, align);
    CHECK(a.ls >= 0 && a.le <= n - 1 && a.ls <= a.le && a.ls % align == 0, "own %d g %d/%d mc %d m0 %d", own, glo,
          ghi, mc, m0);
    CHECK(a.ws >= a.ls && a.we <= a.le, "window outside loaded range");
    for (int m = m0; m < m1; ++m) {
      const int w0 = std::max(0, mc * m - 1 + glo), w1 = std::min(n - 1, mc * m + mc + glo);
      CHECK(w0 >= a.ls && w1 <= a.le, "macrocell %d window [%d, %d] outside [%d, %d]", m, w0, w1, a.ls, a.le);
    }
    for (int v = 0; v < n; ++v) {
      const int anchor = v & ~(align - 1);
      if (anchor >= a.cs && anchor < a.ce) {
        ++writers[v];
        if (v >= a.ls && v <= a.le) ++loaded_by_writer[v];
      }
    }
  }
  for (int v = 0; v < n; ++v) {
    CHECK(writers[v] == 1, "voxel %d written %d times (own %d g %d/%d mc %d align %d per %d)", v, writers[v], own,
          glo, ghi, mc, align, per);
    CHECK(loaded_by_writer[v] == 1, "voxel %d not loaded by its writer", v);
  }
}

static void check_x(int own, int glo, int ghi, int mc) {
  const int n = own + glo + ghi, md = (own + mc - 1) / mc;
  const int spans = (n + dpr::kCmCols - 1) / dpr::kCmCols;
  std::vector<int> p0(md, 0), p1(md, 0), lo(md, n), hi(md, -1), cols(md, 0);
  for (int k = 0; k < spans; ++k) {
    const int x0 = dpr::kCmCols * k, x1 = std::min(n - 1, x0 + dpr::kCmCols - 1);
    const dpr::XCells c = dpr::xspan_cells(k, md, mc, glo, n);
    for (int m = 0; m < md; ++m) {
      const int w0 = std::max(0, mc * m - 1 + glo), w1 = std::min(n - 1, mc * m + mc + glo);
      const bool meets = w0 <= x1 && w1 >= x0;
      CHECK(meets == (m >= c.m0 && m <= c.m1), "span %d lists macrocell %d wrongly (own %d g %d/%d mc %d)", k, m, own,
            glo, ghi, mc);
      if (!meets) continue;
      const int a = std::max(w0, x0), b = std::min(w1, x1);
      lo[m] = std::min(lo[m], a);
      hi[m] = std::max(hi[m], b);
      cols[m] += b - a + 1;
      if (w0 >= x0) {
        ++p0[m];
        if (w1 <= x1) ++p1[m];
      } else {
        ++p1[m];
      }
    }
  }
  for (int m = 0; m < md; ++m) {
    const int w0 = std::max(0, mc * m - 1 + glo), w1 = std::min(n - 1, mc * m + mc + glo);
    CHECK(lo[m] == w0 && hi[m] == w1 && cols[m] == w1 - w0 + 1, "macrocell %d window not covered once", m);
    CHECK(p0[m] == 1 && p1[m] == 1, "macrocell %d partials written %d, %d times (own %d g %d/%d mc %d)", m, p0[m],
          p1[m], own, glo, ghi, mc);
  }
}

static void check_z(int own, int glo, int ghi, int mc, int seg) {
  const int n = own + glo + ghi, md = (own + mc - 1) / mc;
  std::vector<int> writers(n, 0);
  for (int m0 = 0; m0 < md; m0 += seg) {
    const int m1 = std::min(md, m0 + seg);
    // stage in which each row is visited by this segment (-2: not visited)
    std::vector<int> seen(n, -2);
    for (int s = m0 - 1; s <= m1; ++s) {
      const dpr::ZStage st = dpr::z_stage(s, m0, m1, md, mc, glo, n);
      CHECK(st.lo % 2 == 0 && st.lo >= 0 && st.hi <= n + 1, "stage %d [%d, %d)", s, st.lo, st.hi);
      CHECK(st.own == (s >= m0 && s < m1), "stage %d ownership", s);
      for (int zp = st.lo; zp < st.hi; zp += 2) {
        for (int r = zp; r <= zp + 1 && r < n; ++r) {
          CHECK(seen[r] == -2, "row %d visited twice in segment %d", r, m0);
          seen[r] = s;
          if (st.own) ++writers[r];
          for (int m = m0; m < m1; ++m) {
            const int w0 = std::max(0, mc * m - 1 + glo), w1 = std::min(n - 1, mc * m + mc + glo);
            if (r >= w0 && r <= w1)
              CHECK(m >= s - 1 && m <= s + 1, "row %d of stage %d in window of macrocell %d", r, s, m);
          }
        }
      }
    }
    for (int m = m0; m < m1; ++m) {
      const int w0 = std::max(0, mc * m - 1 + glo), w1 = std::min(n - 1, mc * m + mc + glo);
      for (int r = w0; r <= w1; ++r)
        CHECK(seen[r] != -2 && seen[r] <= m + 1, "row %d of macrocell %d window: stage %d (own %d g %d/%d mc %d seg %d)",
              r, m, seen[r], own, glo, ghi, mc, seg);
    }
  }
  for (int r = 0; r < n; ++r)
    CHECK(writers[r] == 1, "row %d written %d times (own %d g %d/%d mc %d seg %d)", r, writers[r], own, glo, ghi, mc,
          seg);
}

int main() {
  std::mt19937 rng(20240700);
  int cases = 0;
  const int edges[] = {2, 4, 8, 16, 32, 64};
  for (int it = 0; it < 4000; ++it) {
    const int mc = edges[rng() % 6];
    const int own = 2 + (int)(rng() % (it < 3000 ? 200 : 2100));
    const int glo = (int)(rng() % 4), ghi = (int)(rng() % 4);
    // x: aligned spans; y: row pairs, one macrocell per span; z: streamed segments
    check_x(own, glo + (it % 7 == 0 ? 150 : 0), ghi, mc);
    check_axis(own, glo, ghi, mc, 2, 1);
    check_z(own, glo, ghi, mc, 1 + (int)(rng() % 12));
    ++cases;
  }
  std::printf("%d cases, %d failures\n", cases, fails);
  return fails ? 1 : 0;
}
