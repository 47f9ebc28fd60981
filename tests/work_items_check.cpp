// Prints the step kernel's work list for a launch shape, as the library builds it, so that
// the CPU tests can check its properties (coverage, strips, segments, order, stream groups).
// stdin:  esize width seg_rows persistent xcd_swizzle streams n, then n lines "nz nr".
// stdout: "group first count" per stream group, then "inst k0 ncols s e" per item in order.
#include <cstdio>
#include <vector>

#include "work_items.h"

int main() {
  int esize, width, seg, persistent, xcd, streams, n;
  if (std::scanf("%d %d %d %d %d %d %d", &esize, &width, &seg, &persistent, &xcd, &streams, &n) != 7) return 2;
  if (streams < 1 || streams > lbm::kMaxStreams || n < 1) return 2;
  std::vector<lbm_axi_params> prm(n);
  for (auto& p : prm)
    if (std::scanf("%d %d", &p.nz, &p.nr) != 2) return 2;
  lbm_axi_launch c{width, seg, persistent, 0, xcd, 0, streams};
  int first[lbm::kMaxStreams] = {}, count[lbm::kMaxStreams] = {};
  const std::vector<lbm::WorkItem> items = lbm::launch_items(prm, esize, c, first, count);
  for (int g = 0; g < streams; ++g) std::printf("%d %d %d\n", g, first[g], count[g]);
  for (const auto& w : items) std::printf("%d %d %d %d %d\n", w.inst, w.k0, w.ncols, w.s, w.e);
  return 0;
}
