// Host check of the one-pass commit's index spans (commit_span.h): for brick
// extents, ghost widths and macrocell edges drawn at random, along one axis
//  - every stored voxel is written by exactly one span (its aligned group's first
//    voxel lies in exactly one core) and that span loads it;
//  - loaded ranges stay inside the stored range, start aligned, and (x) fit the
//    workgroup's column arrays;
//  - every macrocell's window [mc m - 1, mc m + mc] (owned coordinates, clipped)
//    lies inside the loaded range of the span that reduces it.
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
    if (align == 4) CHECK(a.le - a.ls + 1 <= dpr::kCmCols, "x width %d", a.le - a.ls + 1);
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

int main() {
  std::mt19937 rng(20240700);
  int cases = 0;
  const int edges[] = {2, 4, 8, 16, 32, 64};
  for (int it = 0; it < 4000; ++it) {
    const int mc = edges[rng() % 6];
    const int own = 2 + (int)(rng() % (it < 3000 ? 200 : 2100));
    const int glo = (int)(rng() % 4), ghi = (int)(rng() % 4);
    const int n = own + glo + ghi, md = (own + mc - 1) / mc;
    // x: runs of 4, the launcher's chunking; y and z: row pairs, one macrocell per span
    check_axis(own, glo, ghi, mc, 4, dpr::commit_per_chunk(n, glo, md, mc));
    check_axis(own, glo, ghi, mc, 2, 1);
    ++cases;
  }
  std::printf("%d cases, %d failures\n", cases, fails);
  return fails ? 1 : 0;
}
