// Host checks of the rank launches' host logic (built with hipcc as host
// code by tests/test_host_helpers.py):
//  - build_costed_tasks: every (set, strip, row block rb >= 4 g0) of random
//    single sets and batches lies in exactly one task, tasks stay inside
//    their set and strip, the per-XCD queue bounds tile the list, and the
//    list never exceeds max_pair_tasks (the buffer the count reserves);
//  - fix_bits: the fixed-point scale keeps N * max|d| * 2^F below 2^62 (no
//    partial or total can overflow) and within a factor 4 of it.
#include <math.h>
#include <stdio.h>

#include <random>
#include <vector>

#include "worklist.h"

using namespace kd;

static int check_worklists() {
  std::mt19937 rng(1);
  for (int trial = 0; trial < 400; trial++) {
    const uint32_t nsets = 1 + rng() % (trial % 3 == 0 ? 1 : 300);
    std::vector<SetView> views(nsets);
    std::vector<uint32_t> gf(nsets + 1, 0), len;
    for (uint32_t q = 0; q < nsets; q++) {
      const uint32_t N = nsets == 1 ? 1 + rng() % 30000 : 1 + rng() % 2100;
      views[q].N = N;
      views[q].G = (N + 63) / 64;
      gf[q + 1] = gf[q] + views[q].G;
      uint32_t l = 16;
      for (uint32_t g = 0; g < views[q].G; g++) {
        l += 16 * (rng() % 3);
        len.push_back(l);
      }
    }
    const uint32_t tpc = 1u << (rng() % 6);
    const int cus = 1 + (int)(rng() % 300);
    std::vector<PairTask> out;
    uint32_t beg[kXcdQueues + 1];
    build_costed_tasks(views, gf, len, tpc, cus, out, beg);
    if (out.size() > max_pair_tasks(views, tpc, cus)) {
      printf("trial %d: %zu tasks above the bound\n", trial, out.size());
      return 1;
    }
    if (beg[0] != 0 || beg[kXcdQueues] != out.size()) return printf("queue bounds\n"), 1;
    for (uint32_t x = 0; x < kXcdQueues; x++)
      if (beg[x] > beg[x + 1]) return printf("queue order\n"), 1;
    for (const PairTask &t : out)
      if (t.set >= nsets || t.g0 % kGroupsPerTask || t.g0 >= views[t.set].G || t.rb1 <= t.rb0 ||
          t.rb0 < 4 * t.g0 || t.rb1 > (views[t.set].N + 15) / 16)
        return printf("trial %d: bad task\n", trial), 1;
    for (uint32_t q = 0; q < nsets; q++) {
      const uint32_t RB = (views[q].N + 15) / 16;
      for (uint32_t g0 = 0; g0 < views[q].G; g0 += kGroupsPerTask) {
        std::vector<int> seen(RB, 0);
        for (const PairTask &t : out)
          if (t.set == q && t.g0 == g0)
            for (uint32_t rb = t.rb0; rb < t.rb1; rb++) seen[rb]++;
        for (uint32_t rb = 0; rb < RB; rb++)
          if (seen[rb] != (rb >= 4 * g0 ? 1 : 0)) {
            printf("trial %d: set %u strip %u row block %u covered %d times\n", trial, q, g0, rb, seen[rb]);
            return 1;
          }
      }
    }
  }
  printf("work lists: 400 random sets and batches covered exactly\n");
  return 0;
}

static int check_fix_bits() {
  std::mt19937_64 g(3);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int i = 0; i < 200000; i++) {
    const uint32_t n = 1 + (uint32_t)(u(g) * (i % 2 ? 1e4 : 2e8));
    const double delta = pow(10.0, -300.0 + 600.0 * u(g));
    const int F = fix_bits(n, delta);
    const double dmax = fmax(fabs(log(delta)), log1p(delta));
    const double bound = ldexp((double)n * dmax, F);
    if (!(bound < ldexp(1.0, 62)) || !(bound >= ldexp(1.0, 60))) {
      printf("fix_bits(%u, %g) = %d: bound %g\n", n, delta, F, bound);
      return 1;
    }
    // every d = -ln(delta + f), 0 <= f <= 1, is within dmax
    for (double f : {0.0, 0.5, 1.0})
      if (fabs(-log(delta + f)) > dmax * (1 + 1e-15)) return printf("dmax\n"), 1;
  }
  printf("fix_bits: 200000 (N, delta) scales within 2^60 .. 2^62\n");
  return 0;
}

int main() {
  if (check_worklists() || check_fix_bits()) return 1;
  printf("OK\n");
  return 0;
}
