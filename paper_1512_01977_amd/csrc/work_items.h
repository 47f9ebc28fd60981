// Work lists of the fused step kernel, built on the host: strips of output columns times
// row segments, their order over the XCDs, and the split of a batch into stream groups.
// Plain host code (no HIP calls), shared by the library and its CPU tests.
#pragma once

#include <algorithm>
#include <vector>

#include "lbm_axi.h"
#include "lbm_axi_internal.h"

namespace lbm {

constexpr int kMaxStreams = 4;  // stream groups of one handle
constexpr int kXcds = 8;        // XCDs that a launch's workgroups are dealt over, b % 8

// Work-item count and lane-iterations of a launch shape (cost model of the default shape).
inline void shape_cost(const std::vector<lbm_axi_params>& prm, int esize, int width, int seg, long long* items,
                       long long* lane_iters, int* longest) {
  *items = 0;
  *lane_iters = 0;
  *longest = 0;
  const int wout = strip_cols(width, esize);
  for (const auto& p : prm) {
    const int sg = std::min(seg > 0 ? std::min(seg, p.nr) : p.nr, max_item_rows(row_pitch(p.nz, esize), esize));
    const long long nstrip = std::max(1, (p.nz + wout - 1) / wout);
    const long long nseg = (p.nr + sg - 1) / sg;
    const int rows = sg + std::min(12, p.nr - sg + 12);  // segment plus its pipeline rows
    *items += nstrip * nseg;
    *lane_iters += nstrip * nseg * (long long)width * rows;
    *longest = std::max(*longest, rows);
  }
}

// Reorder a longest-first item list for a launch of one workgroup per item.  The hardware
// hands workgroup b to XCD b % 8, and each XCD has its own L2.  Neighbouring strips of one
// row band (same instance, same segment) read each other's edge lines, so the strips of a
// band go to one XCD, where they run at about the same time and the shared lines come from
// its L2 instead of HBM.  Bands are dealt in order to the XCD with the most room left; each
// XCD keeps the list's longest-first order, and XCD x receives exactly the items at
// positions x, x + 8, ... (a band that does not fit in the room left is split).
inline std::vector<WorkItem> deal_over_xcds(const std::vector<WorkItem>& items) {
  const size_t n = items.size();
  std::vector<WorkItem> per[kXcds];
  size_t room[kXcds];
  for (int x = 0; x < kXcds; ++x) room[x] = n / kXcds + ((size_t)x < n % kXcds ? 1 : 0);
  for (size_t i = 0; i < n;) {
    size_t j = i + 1;
    while (j < n && items[j].inst == items[i].inst && items[j].s == items[i].s) ++j;
    while (i < j) {
      int x = 0;
      for (int y = 1; y < kXcds; ++y)
        if (room[y] > room[x]) x = y;
      const size_t take = std::min(room[x], j - i);
      per[x].insert(per[x].end(), items.begin() + i, items.begin() + i + take);
      room[x] -= take;
      i += take;
    }
  }
  std::vector<WorkItem> out(n);
  for (int x = 0; x < kXcds; ++x)
    for (size_t k = 0; k < per[x].size(); ++k) out[k * kXcds + x] = per[x][k];
  return out;
}

// Strips of whole 128-byte lines of output columns (at most width - 12) times row
// segments, for the instances k with keep[k] != 0 (every instance when keep is empty).
inline std::vector<WorkItem> build_items(const std::vector<lbm_axi_params>& prm, int esize, const lbm_axi_launch& c,
                                         const std::vector<char>& keep) {
  std::vector<WorkItem> items;
  const int wout = strip_cols(c.width, esize);
  for (int k = 0; k < (int)prm.size(); ++k) {
    if (!keep.empty() && !keep[k]) continue;
    const auto& p = prm[k];
    const int seg = std::min(c.seg_rows > 0 ? c.seg_rows : p.nr, max_item_rows(row_pitch(p.nz, esize), esize));
    const int nstrip = std::max(1, (p.nz + wout - 1) / wout);
    for (int s = 0; s < p.nr; s += seg)
      for (int q = 0; q < nstrip; ++q) {
        WorkItem w;
        w.inst = k;
        w.k0 = q * wout;
        w.ncols = std::min(wout, p.nz - w.k0);
        w.s = s;
        w.e = std::min(p.nr, s + seg);
        items.push_back(w);
      }
  }
  if (c.persistent || c.xcd_swizzle != 1) {
    // longest first (rows swept, halo included), so the queue drains evenly; without the
    // XCD swizzle the hardware deals consecutive workgroups round-robin over the XCDs, so
    // the same order balances a one-item-per-workgroup launch too
    auto cost = [](const WorkItem& w) { return (w.e - w.s) + std::min(6, w.s) + 6; };
    std::stable_sort(items.begin(), items.end(),
                     [&](const WorkItem& a, const WorkItem& b) { return cost(a) > cost(b); });
    if (!c.persistent && c.xcd_swizzle == 2) return deal_over_xcds(items);
  }
  return items;
}

// The group of each instance: largest instances first, each to the group with the fewest
// nodes so far (every group gets at least one instance when groups <= n).
inline std::vector<int> group_of_instances(const std::vector<lbm_axi_params>& prm, int groups) {
  const int n = (int)prm.size();
  std::vector<int> order(n), grp(n, 0);
  for (int k = 0; k < n; ++k) order[k] = k;
  auto nodes = [&](int k) { return (long long)prm[k].nz * prm[k].nr; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nodes(a) > nodes(b); });
  long long load[kMaxStreams] = {};
  for (int k : order) {
    int g = 0;
    for (int x = 1; x < groups; ++x)
      if (load[x] < load[g]) g = x;
    grp[k] = g;
    load[g] += nodes(k);
  }
  return grp;
}

// The work list of a launch shape: each stream group's items, one group after the other
// (group g owns first[g] .. first[g] + count[g] - 1).  c.streams must be 1 .. kMaxStreams.
inline std::vector<WorkItem> launch_items(const std::vector<lbm_axi_params>& prm, int esize, const lbm_axi_launch& c,
                                          int first[kMaxStreams], int count[kMaxStreams]) {
  const std::vector<int> grp = group_of_instances(prm, c.streams);
  std::vector<WorkItem> all;
  for (int g = 0; g < c.streams; ++g) {
    std::vector<char> keep(prm.size());
    for (size_t k = 0; k < prm.size(); ++k) keep[k] = grp[k] == g;
    const std::vector<WorkItem> items = build_items(prm, esize, c, keep);
    first[g] = (int)all.size();
    count[g] = (int)items.size();
    all.insert(all.end(), items.begin(), items.end());
  }
  return all;
}

}  // namespace lbm
