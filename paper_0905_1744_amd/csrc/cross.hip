// Globalized k-mer rank, the cross pass (paper Section 3.1.1; Algorithm 2
// step 6): every sequence of a counted batch of blocks against the samples
// gathered from all blocks, with the tile machinery of the all-pairs rank
// kernel (tile.h).
#include <algorithm>
#include <vector>

#include "tile.h"

namespace kd {

// Globalized rank, step 6 of Algorithm 2 (Section 3.1.1): every sequence of
// the counted blocks (columns, all sets of `cols`) against the gathered
// samples (rows: the single set *rows).  One workgroup = gpt (16 or 32)
// column groups of the whole batch, gperm[gx0 .. gx0+gpt-1], against sample
// row blocks rb0 .. rb1-1.  gperm lists the groups by decreasing list
// length, so the groups of a workgroup are about equally long; wave w takes
// the w-th of them and, with 32, also the (31-w)-th.  Each group belongs to
// whichever set holds it.
// Each pair adds d(column, sample) to the column's exact accumulator;
// nothing is added for the rows.
// set and set-local index of batch-wide column group gx (wave-uniform)
__device__ __forceinline__ uint32_t cross_set(const Segs &cols, uint32_t gx, uint32_t &gl) {
  const uint32_t q = __builtin_amdgcn_readfirstlane(cols.set_of_grp(gx));
  gl = gx - __builtin_amdgcn_readfirstlane(cols.grp[q]);
  return q;
}

__global__ __launch_bounds__(1024) void rank_cross_kernel(Segs cols, const SetView *__restrict__ rows,
                                                          const CrossTask *__restrict__ tasks,
                                                          const uint32_t *__restrict__ gperm,
                                                          uint32_t gpt, double delta) {
  __shared__ RankShared sh;
  const CrossTask tk = tasks[blockIdx.x];
  const SetView rv = *rows;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (uint32_t q = tid; q < (uint32_t)kLogEntries; q += 1024) log_table_entry((int)q, sh.logt[q]);
  if (tid == 0) sh.ln2 = log(2.0);
  clear_rows(sh.row);
  const int fix = fix_bits(rv.N, delta);

  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t ga = __builtin_amdgcn_readfirstlane(gperm[tk.gx0 + wave]);
  const uint32_t gb = gpt == 32u ? __builtin_amdgcn_readfirstlane(gperm[tk.gx0 + 31u - wave]) : kNone;
  sh.colacc[wave][lane] = 0;
  sh.colacc[31u - wave][lane] = 0;

  for (uint32_t rb = tk.rb0; rb < tk.rb1; rb++) {
    if (rb > tk.rb0) {
      const uint32_t pr = rb - 1;
      touch_rows<false>(rv, ConsecutiveRows{16u * pr, rv.N}, rv.exc_ids, rv.exc_off[pr], rv.exc_n[pr], sh.row);
    }
    __syncthreads();
    const uint32_t e0 = rv.exc_off[rb], en = rv.exc_n[rb];
    touch_rows<true>(rv, ConsecutiveRows{16u * rb, rv.N}, rv.exc_ids, e0, en, sh.row);
    const bool lds_exc = en <= kExcLds;
    if (lds_exc) {
      for (uint32_t e = tid; e < 16u * en; e += 1024) sh.exc_c[e] = rv.exc_cnt[16ull * e0 + e];
    }
    __syncthreads();
    const uint16_t *ecnt = lds_exc ? sh.exc_c : rv.exc_cnt + 16ull * e0;
    if (ga != kNone) {
      uint32_t gl;
      const uint32_t q = cross_set(cols, ga, gl);
      rank_tile<true>(cols.views[q], sh, rb, gl, rv.N, delta, fix, ecnt, sh.colacc[wave]);
    }
    if (gb != kNone) {
      uint32_t gl;
      const uint32_t q = cross_set(cols, gb, gl);
      rank_tile<true>(cols.views[q], sh, rb, gl, rv.N, delta, fix, ecnt, sh.colacc[31u - wave]);
    }
    __syncthreads();
  }
#pragma unroll
  for (uint32_t h = 0; h < 2; h++) {
    const uint32_t gx = h ? gb : ga;
    if (gx == kNone) continue;
    uint32_t gl;
    const SetView &v = cols.views[cross_set(cols, gx, gl)];
    const uint32_t sc = 64u * gl + lane;
    if (sc < v.N)
      atomicAdd(reinterpret_cast<unsigned long long *>(v.acc) + sc,
                (unsigned long long)sh.colacc[h ? 31u - wave : wave][lane]);
  }
}

hipError_t launch_rank_cross(hipStream_t st, const Segs &cols, const SetView *rows,
                             const CrossTask *tasks, uint32_t ntasks, const uint32_t *gperm,
                             uint32_t gpt, double delta) {
  if (ntasks == 0) return hipSuccess;
  if (gpt != 16u && gpt != 32u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rank_cross_kernel, dim3(ntasks), dim3(1024), 0, st, cols, rows, tasks, gperm,
                     gpt, delta);
  return hipGetLastError();
}

// Globalized rank = (sum over the S samples) / S for every sorted position
// of every block, written at the input index; clears the accumulators.
__global__ void cross_finalize_kernel(Segs sg, uint32_t N, uint32_t S, double delta,
                                      double *__restrict__ ranks) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const uint32_t set = sg.set_of_pos(p);
  const uint32_t a = sg.seq[set];
  const SetView &v = sg.views[set];
  long long *acc = v.acc + (p - a);
  ranks[a + v.perm[p - a]] = fix_value(*acc, fix_bits(S, delta)) / (double)S;
  *acc = 0;
}

hipError_t launch_cross_finalize(hipStream_t st, const Segs &sg, uint32_t N, uint32_t S,
                                 double delta, double *ranks) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(cross_finalize_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sg, N, S,
                     delta, ranks);
  return hipGetLastError();
}

// Work list of the globalized-rank pass.
//  * The column groups of all sets are ordered by decreasing padded list
//    length (grp_len, read back from the device; ties by group number) into
//    gperm, and consecutive runs of `gpt` of them form the strips, so the
//    groups a workgroup's waves walk together are about equally long.
//    gpt = 32 (two groups per wave) unless that leaves fewer than two
//    workgroups per compute unit, then 16 (one group per wave).
//  * Each strip is cut into at most one XCD's worth of runs of sample row
//    blocks.
//  * Placement: workgroup t runs on XCD t % 8 and an XCD starts its
//    workgroups in order as its compute units free up.  Tasks, longest
//    first, are assigned to the XCD whose next free compute unit (in a
//    simulation with a cost of rows x list length per task) frees first,
//    ties to the lowest XCD, so consecutive tasks of one strip tend to
//    share an XCD and its L2; the list then interleaves the XCDs' queues.
//    Positions past an XCD's queue hold empty tasks (no row blocks, no
//    groups).
// gperm gets gpt (strips + 1) entries, 0xFFFFFFFF past the last group.
constexpr uint32_t kXcds = 8;

uint32_t make_cross_tasks(const uint32_t *grp_len, uint32_t Gtot, uint32_t RBs, int cus,
                          std::vector<CrossTask> &out, std::vector<uint32_t> &gperm) {
  out.clear();
  const uint32_t ncu = (uint32_t)std::max(cus, (int)kXcds);
  const uint32_t per_xcd = ncu / kXcds;
  const uint32_t runs = std::max<uint32_t>(1, std::min(RBs, per_xcd));
  const uint32_t rbt = (RBs + runs - 1) / runs;
  const uint32_t nrun = (RBs + rbt - 1) / rbt;
  uint32_t gpt = kGroupsPerTask;
  if ((uint64_t)((Gtot + 31) / 32) * nrun < 2ull * ncu) gpt = kGroupsPerTask / 2;
  const uint32_t strips = (Gtot + gpt - 1) / gpt;
  gperm.assign((size_t)(strips + 1) * gpt, 0xFFFFFFFFu);
  for (uint32_t g = 0; g < Gtot; g++) gperm[g] = g;
  std::stable_sort(gperm.begin(), gperm.begin() + Gtot,
                   [&](uint32_t a, uint32_t b) { return grp_len[a] > grp_len[b]; });
  // per-XCD min-heaps of compute-unit free times
  std::vector<std::vector<uint64_t>> cu(kXcds, std::vector<uint64_t>(per_xcd, 0));
  std::vector<std::vector<CrossTask>> per(kXcds);
  auto later = [](uint64_t a, uint64_t b) { return a > b; };
  for (uint32_t s = 0; s < strips; s++) {
    const uint32_t g0 = s * gpt;
    // the wave with the most work: groups w and gpt-1-w (gpt = 32) or w
    uint64_t wmax = 0;
    for (uint32_t w = 0; w < 16; w++) {
      uint64_t l = gperm[g0 + w] != 0xFFFFFFFFu ? grp_len[gperm[g0 + w]] : 0;
      if (gpt == 32 && gperm[g0 + 31 - w] != 0xFFFFFFFFu) l += grp_len[gperm[g0 + 31 - w]];
      wmax = std::max(wmax, l);
    }
    for (uint32_t rb0 = 0; rb0 < RBs; rb0 += rbt) {
      const uint32_t rb1 = std::min(rb0 + rbt, RBs);
      const uint64_t cost = (uint64_t)(rb1 - rb0) * (wmax + 64);
      uint32_t bx = 0;
      for (uint32_t x = 1; x < kXcds; x++)
        if (cu[x].front() < cu[bx].front()) bx = x;
      std::pop_heap(cu[bx].begin(), cu[bx].end(), later);
      cu[bx].back() += cost;
      std::push_heap(cu[bx].begin(), cu[bx].end(), later);
      per[bx].push_back({g0, rb0, rb1});
    }
  }
  size_t L = 0;
  for (const auto &v : per) L = std::max(L, v.size());
  out.assign(L * kXcds, CrossTask{strips * gpt, 0, 0});
  for (uint32_t x = 0; x < kXcds; x++)
    for (size_t j = 0; j < per[x].size(); j++) out[j * kXcds + x] = per[x][j];
  return gpt;
}

}  // namespace kd
