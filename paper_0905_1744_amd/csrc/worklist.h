// Host-side work lists of the all-pairs kernels (no device code): which
// tasks (runs of row blocks against strips of 32 column groups) a launch
// runs, and in which per-XCD queue.  Included by kd_api.hip and by the host
// test tests/host/worklist_check.cpp.
#pragma once

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "kd_internal.h"

namespace kd {

// Plain work list of one set of N sequences: strips of 32 column groups
// (two per wave of a workgroup) against runs of `rbt` row blocks; a row
// block rb only meets column groups g <= rb/4 (pairs below the diagonal of
// the sorted order).  Largest first.  (The distance-matrix pass, which has
// no accumulators to flush, uses it with one row block per workgroup.)
inline void make_tasks(uint32_t N, uint32_t set_index, uint32_t rbt, std::vector<PairTask> &out) {
  std::vector<PairTask> t;
  const uint32_t RB = (N + 15) / 16, G = (N + 63) / 64;
  for (uint32_t g0 = 0; g0 < G; g0 += kGroupsPerTask) {
    for (uint32_t rb0 = 4u * g0; rb0 < RB; rb0 += rbt)
      t.push_back({set_index, rb0, std::min(rb0 + rbt, RB), g0});
  }
  std::stable_sort(t.begin(), t.end(), [](const PairTask &a, const PairTask &b) {
    if (a.g0 != b.g0) return a.g0 > b.g0;
    return a.rb1 - a.rb0 > b.rb1 - b.rb0;
  });
  out.insert(out.end(), t.begin(), t.end());
}

// number of 16 x 64 tiles of a task (its share of the triangle)
inline uint64_t task_tiles(const PairTask &t, uint32_t G) {
  uint64_t n = 0;
  const uint32_t g1 = std::min(t.g0 + kGroupsPerTask, G);
  for (uint32_t rb = t.rb0; rb < t.rb1; rb++) {
    const uint32_t gmax = rb / 4;  // groups g <= rb/4 are active
    if (gmax >= t.g0) n += std::min(gmax + 1, g1) - t.g0;
  }
  return n;
}

inline void build_task_list(const std::vector<SetView> &views, uint32_t rbt, std::vector<PairTask> &out) {
  out.clear();
  for (uint32_t q = 0; q < views.size(); q++) make_tasks(views[q].N, q, rbt, out);
  if (views.size() > 1) {
    std::vector<std::pair<uint64_t, uint32_t>> key(out.size());
    for (size_t t = 0; t < key.size(); t++) key[t] = {task_tiles(out[t], views[out[t].set].G), (uint32_t)t};
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint64_t, uint32_t> &a,
                        const std::pair<uint64_t, uint32_t> &b) { return a.first > b.first; });
    std::vector<PairTask> sorted(key.size());
    for (size_t t = 0; t < key.size(); t++) sorted[t] = out[key[t].second];
    out.swap(sorted);
  }
}

// Cost model of the rank kernel, in units of one 32-word lookup step of a
// wave: a tile (row block, column group) costs its group's padded list
// length / 32 plus kTileCost (counts transpose, FP64 epilogue, flushes); a
// row block of a strip costs the busiest wave's tiles (wave w holds groups
// g0 + w and g0 + 31 - w) plus kRowBlockCost (table fill and clear, two
// barriers).
constexpr double kTileCost = 4.0;
constexpr double kRowBlockCost = 6.0;

// Rank work list of every set of a counted object.
//  - The row blocks of all strips (32 column groups) of all sets, strip
//    after strip, form one sequence of units with an estimated cost.  It is
//    cut into 8 contiguous pieces of equal cost, one per XCD, so that the
//    strips an XCD works on (their column lists) stay in its own L2.
//  - Each piece is cut into about T / 8 runs of equal cost (T = tasks_per_cu
//    x compute units), never across a strip: fewer, longer runs flush fewer
//    column sums (one 64-bit atomic per column per workgroup), more runs
//    balance better.
//  - The pieces become the per-XCD queues of the persistent rank launch
//    (out[beg[x] .. beg[x+1]), largest first); a workgroup takes from its
//    own XCD's queue and steals from the others once it is empty.  (Kept in
//    strip order instead, the 20k launch took 1.28 ms instead of 1.23 and
//    fetched no fewer bytes.)  "Largest first" is a stable counting sort on
//    the cost quantized to kCostLevels levels of the largest task: it runs
//    in linear time while the device lays the lists out.
//  - In a batch the key is the set's whole cost, so that a set's runs stay
//    together in its queue and the compute units that take them at about
//    the same time share its column lists in the XCD's L2 (ordered by the
//    runs' own costs, every unit of an XCD worked on a set of its own and
//    the 4,096-set launch fetched 36 GB).
// grp_len: host copy of every column group's padded list length
// (batch-wide numbering).
constexpr uint32_t kCostLevels = 1024;

inline void build_costed_tasks(const std::vector<SetView> &views, const std::vector<uint32_t> &grp_first,
                               const std::vector<uint32_t> &grp_len, uint32_t tasks_per_cu, int cus,
                               std::vector<PairTask> &out, uint32_t (&beg)[kXcdQueues + 1]) {
  out.clear();
  for (uint32_t x = 0; x <= kXcdQueues; x++) beg[x] = 0;
  struct Strip { uint32_t set, g0, rb0, rb1; };
  std::vector<Strip> strips;
  std::vector<double> cost;
  size_t nunits = 0;
  for (const SetView &w : views) nunits += (w.N + 15) / 16 * (size_t)(((w.N + 63) / 64 + kGroupsPerTask - 1) / kGroupsPerTask);
  cost.reserve(nunits);
  double all = 0.0;
  for (uint32_t q = 0; q < views.size(); q++) {
    const uint32_t N = views[q].N, RB = (N + 15) / 16, G = (N + 63) / 64;
    const uint32_t *L = grp_len.data() + grp_first[q];
    for (uint32_t g0 = 0; g0 < G; g0 += kGroupsPerTask) {
      double wave_cost[16] = {0.0};
      double worst = 0.0;
      if (4u * g0 < RB) strips.push_back({q, g0, 4u * g0, RB});
      for (uint32_t rb = 4u * g0; rb < RB; rb++) {
        if ((rb & 3u) == 0) {  // group rb / 4 starts to meet the row blocks
          const uint32_t g = rb >> 2;
          if (g < G && g < g0 + kGroupsPerTask) {
            const uint32_t j = g - g0, w = j < 16 ? j : 31u - j;
            wave_cost[w] += L[g] / 32.0 + kTileCost;
            worst = std::max(worst, wave_cost[w]);
          }
        }
        cost.push_back(worst + kRowBlockCost);
        all += worst + kRowBlockCost;
      }
    }
  }
  if (cost.empty()) return;
  const double T = std::max<double>(kXcdQueues, (double)tasks_per_cu * (double)std::max(cus, 1));
  const double per_task = all / T, per_xcd = all / kXcdQueues;
  std::vector<PairTask> tk[kXcdQueues];
  std::vector<double> tc[kXcdQueues];
  for (uint32_t x = 0; x < kXcdQueues; x++) {
    tk[x].reserve((size_t)(T / kXcdQueues) + strips.size() / kXcdQueues + 8);
    tc[x].reserve((size_t)(T / kXcdQueues) + strips.size() / kXcdQueues + 8);
  }
  double cum = 0.0, tcost = 0.0, cmax = 0.0;
  uint32_t xcd = 0;
  // the next XCD boundary, a hair low: the exact test divides only near it
  double thr = per_xcd * (1.0 - 1e-9);
  size_t i = 0;
  for (const Strip &st : strips) {
    uint32_t start = st.rb0;
    for (uint32_t rb = st.rb0; rb < st.rb1; rb++, i++) {
      tcost += cost[i];
      cum += cost[i];
      uint32_t next_xcd = xcd;
      if (cum >= thr) next_xcd = std::min<uint32_t>(kXcdQueues - 1, (uint32_t)(cum / per_xcd));
      if (rb + 1 == st.rb1 || tcost >= per_task || next_xcd != xcd) {
        tk[xcd].push_back(PairTask{st.set, start, rb + 1, st.g0});
        tc[xcd].push_back(tcost);
        cmax = std::max(cmax, tcost);
        start = rb + 1;
        tcost = 0.0;
        if (next_xcd != xcd) {
          xcd = next_xcd;
          thr = per_xcd * (double)(xcd + 1) * (1.0 - 1e-9);
        }
      }
    }
  }
  // levels: kCostLevels, fewer for short queues (a finer grid than the
  // tasks per queue changes nothing but the time to clear it)
  uint32_t levels = 16;
  while (levels < kCostLevels && levels < 4 * (uint32_t)(i / kXcdQueues + 1)) levels *= 2;
  levels = std::min(levels, kCostLevels);
  if (views.size() > 1) {
    // several sets: order by the set's whole cost instead, so that a set's
    // runs stay together (stable sort: in row-block order) and the compute
    // units of an XCD that take them at about the same time share the
    // set's column lists in L2
    std::vector<double> scost(views.size(), 0.0);
    for (uint32_t x = 0; x < kXcdQueues; x++)
      for (size_t k = 0; k < tk[x].size(); k++) scost[tk[x][k].set] += tc[x][k];
    cmax = 0.0;
    for (uint32_t x = 0; x < kXcdQueues; x++)
      for (size_t k = 0; k < tk[x].size(); k++) {
        tc[x][k] = scost[tk[x][k].set];
        cmax = std::max(cmax, tc[x][k]);
      }
  }
  const double scale = cmax > 0.0 ? (levels - 1) / cmax : 0.0;
  std::vector<uint32_t> cnt(levels + 1);
  std::vector<uint16_t> key;
  out.reserve(i);
  for (uint32_t x = 0; x < kXcdQueues; x++) {
    const std::vector<double> &c = tc[x];
    std::fill(cnt.begin(), cnt.end(), 0u);
    key.resize(c.size());
    for (size_t k = 0; k < c.size(); k++) {
      const uint32_t lv = std::min(levels - 1, (uint32_t)(c[k] * scale));
      key[k] = (uint16_t)(levels - 1 - lv);
      cnt[key[k] + 1u]++;
    }
    for (uint32_t q = 0; q < levels; q++) cnt[q + 1] += cnt[q];
    beg[x] = (uint32_t)out.size();
    out.resize(out.size() + c.size());
    PairTask *o = out.data() + beg[x];
    for (size_t k = 0; k < c.size(); k++) o[cnt[key[k]]++] = tk[x][k];
  }
  beg[kXcdQueues] = (uint32_t)out.size();
}

// Most tasks build_costed_tasks can make: a run ends when its cost reaches
// the per-task share (at most T such runs), at a strip's end or at an XCD
// boundary.
inline uint64_t max_pair_tasks(const std::vector<SetView> &views, uint32_t tasks_per_cu, int cus) {
  uint64_t strips = 0;
  for (const SetView &w : views) strips += ((w.N + 63) / 64 + kGroupsPerTask - 1) / kGroupsPerTask;
  const uint64_t T = std::max<uint64_t>(kXcdQueues, (uint64_t)tasks_per_cu * (uint64_t)std::max(cus, 1));
  return T + strips + kXcdQueues + 1;
}

}  // namespace kd
