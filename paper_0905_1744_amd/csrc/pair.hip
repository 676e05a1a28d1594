// All-pairs shared k-mer counts and the k-mer rank (paper Section 3,
// Equations 1-3).
//
// shared(X,Y) = sum over words of min(cX, cY).  Writing min(a,b) as the
// number of levels t >= 1 with a >= t and b >= t, the t = 1 level is the
// size of the intersection of the two word sets and the higher levels only
// involve words present at least twice in both sequences.
//
// Level 1.  A workgroup owns a row block of 16 sequences and builds in LDS a
// 46656-entry table of 16-bit masks: bit r of entry w says row r holds word
// w.  Each wave then streams a group of 64 column sequences (one per lane,
// interleaved layout, 16-byte coalesced loads) and looks every column word
// up once: the mask answers all 16 rows at once.  Two looked-up masks form a
// 32-bit word whose bits are 32 independent one-bit counters; the words are
// summed with carry-save adders (Harley-Seal) into bit planes, so a 32-bit
// logic operation advances 32 counters.  At the end of the column list the
// 16 planes are transposed into per-row counts.
//
// Higher levels.  A row block also carries the sorted words that some of
// its rows hold at least twice, with the 16 counts, and a 46656-bit LDS
// bitmap of them.  A column's own count>=2 words are checked against the
// bitmap; on a hit, row r gains max(0, min(c_r, c_col) - 1).
//
// Ranks.  For each pair the fused epilogue forms F = shared / (min(n,m) - 5)
// (Equation 1) and d = -ln(delta + F) (Equation 2) in FP64; the 16x64 tile
// reduces d per row (fixed butterfly) and per column (fixed row order) and
// adds the partial sums to the rows' and columns' accumulators as 64-bit
// fixed-point integers (fix_bits).  Integer addition is associative, so R_i
// (Equation 3) is independent of tiling, scheduling and co-running work.  Each unordered pair is computed once (column position
// below row position in the sorted order), and the j = i term is added by
// the finalize kernel.
#include "tile.h"

namespace kd {

// One task = 16 waves x 2 = 32 consecutive column groups g0..g0+31 (wave w
// takes g0 + w and g0 + 31 - w: lists grow with g, so every wave gets about
// the same total length) against row blocks rb0..rb1-1, one row block at a
// time.  Row partials of a row block meet in LDS (exact integer adds) and
// go to HBM once; column partials stay in LDS across the row blocks and go
// to HBM once at the end of the task.  On entry the table is empty; on
// exit it is empty again.
__device__ __forceinline__ void run_pair_task(const SetView &v, const PairTask &tk, RankShared &sh,
                                              double delta) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int fix = fix_bits(v.N, delta);
  const uint32_t ja = wave, jb = 31u - wave;  // the wave's groups in the strip
  const uint32_t ga = tk.g0 + ja, gb = tk.g0 + jb;
  if (tid < 16) sh.racc[tid] = 0;
  sh.colacc[ja][lane] = 0;
  sh.colacc[jb][lane] = 0;
  // lists of the first group: a strip whose row blocks meet few groups only
  // splits them over several waves when each slice keeps >= kSplitMinWords
  const uint32_t Lfirst = __builtin_amdgcn_readfirstlane(v.grp_len[tk.g0]);

  for (uint32_t rb = tk.rb0; rb < tk.rb1; rb++) {
    if (rb > tk.rb0) {
      // previous row block: flush its row sums, then remove it from the table
      const uint32_t pr = rb - 1;
      if (tid < 16) {
        const uint32_t s = 16u * pr + tid;
        if (s < v.N) atomicAdd(reinterpret_cast<unsigned long long *>(v.acc) + s, sh.racc[tid]);
        sh.racc[tid] = 0;
      }
      touch_rows<false>(v, ConsecutiveRows{16u * pr, v.N}, v.exc_ids, v.exc_off[pr], v.exc_n[pr], sh.row);
    }
    __syncthreads();
    const uint32_t e0 = v.exc_off[rb], en = v.exc_n[rb];
    touch_rows<true>(v, ConsecutiveRows{16u * rb, v.N}, v.exc_ids, e0, en, sh.row);
    const bool lds_exc = en <= kExcLds;
    if (lds_exc) {
      for (uint32_t e = tid; e < 16u * en; e += 1024) sh.exc_c[e] = v.exc_cnt[16ull * e0 + e];
    }
    __syncthreads();
    const uint16_t *ecnt = lds_exc ? sh.exc_c : v.exc_cnt + 16ull * e0;
    // a tile has pairs below the diagonal only when rb >= 4 g: the strip's
    // groups g0 .. g0 + nact - 1 meet this row block
    const uint32_t glast = min(min(tk.g0 + 31u, v.G - 1u), rb >> 2);
    const uint32_t nact = glast + 1u - tk.g0;  // tasks start at rb >= 4 g0
    // Few groups: k waves per group, each counting a 16-word-aligned slice
    // of the group's lists; the counts meet in LDS and the group's first
    // wave finishes the tile with the same arithmetic as a whole tile.
    // Otherwise every wave takes its two groups whole.
    const uint32_t kmax = nact <= 16u ? 16u / nact : 1u;
    const uint32_t k = min(kmax, max(1u, Lfirst / kSplitMinWords));
    const bool split = k > 1u;
    const uint32_t part = wave % k;
#pragma nounroll
    for (uint32_t it = 0; it < (split ? 1u : 2u); it++) {
      const uint32_t j = split ? wave / k : (it ? jb : ja);
      const uint32_t g = tk.g0 + j;
      const bool has = split ? j < nact : (g < v.G && rb >= 4u * g);
      const bool owner = has && part == 0;
      uint32_t cnt[16];
      TileCol tc;
      if (owner) tc = tile_col(v, g);
      if (has) {
        const uint32_t Lq = __builtin_amdgcn_readfirstlane(v.grp_len[g]) >> 4;
        const uint32_t a = 16u * (part * Lq / k), b = 16u * ((part + 1u) * Lq / k);
        if (b > a) {
          slice_counts(v, sh, g, a, b - a, cnt);
        } else {
#pragma unroll
          for (int r = 0; r < 16; r++) cnt[r] = 0u;
        }
        if (!owner) {
#pragma unroll
          for (int r = 0; r < 16; r++) sh.xcnt[wave][r][lane] = (uint16_t)cnt[r];
        }
      }
      if (split) {
        __syncthreads();
        if (owner) {
          for (uint32_t q = 1; q < k; q++) {
#pragma unroll
            for (int r = 0; r < 16; r++) cnt[r] += sh.xcnt[wave + q][r][lane];
          }
        }
      }
      if (owner) tile_finish<false>(v, sh, rb, g, v.N, delta, fix, ecnt, tc, cnt, sh.colacc[j]);
    }
    __syncthreads();
  }
  // last row block: row sums out, rows out of the table; column sums out
  const uint32_t pr = tk.rb1 - 1;
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(v.acc);
  if (tid < 16) {
    const uint32_t s = 16u * pr + tid;
    if (s < v.N) atomicAdd(acc + s, sh.racc[tid]);
  }
  touch_rows<false>(v, ConsecutiveRows{16u * pr, v.N}, v.exc_ids, v.exc_off[pr], v.exc_n[pr], sh.row);
#pragma unroll
  for (uint32_t gi = 0; gi < 2; gi++) {
    const uint32_t g = gi ? gb : ga, sc = 64u * g + lane;
    if (g < v.G && sc < v.N && tk.rb1 > 4u * g)
      atomicAdd(acc + sc, (unsigned long long)sh.colacc[gi ? jb : ja][lane]);
  }
  __syncthreads();
}

// Next task for a workgroup on XCD `home`: from its own XCD's queue while it
// lasts, then from the others in turn; kNoTask when all are empty.
constexpr uint32_t kNoTask = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t take_task(const TaskQueues &q, uint32_t home, uint32_t &empty) {
  for (uint32_t i = 0; i < kXcdQueues; i++) {
    const uint32_t x = (home + i) % kXcdQueues;
    if ((empty >> x) & 1u) continue;
    const uint32_t n = q.beg[x + 1] - q.beg[x];
    const uint32_t t = n ? atomicAdd(q.head + x, 1u) : n;
    if (t < n) return q.beg[x] + t;
    empty |= 1u << x;
  }
  return kNoTask;
}

// Persistent launch: one workgroup per compute unit; each takes tasks from
// the queue of the XCD it runs on (hardware register XCC_ID), so the strips
// an XCD works on keep their column lists in its L2, and steals from the
// other queues when its own is empty.  Every task is taken exactly once
// (one atomic per take); a workgroup exits when all queues are empty.
__global__ __launch_bounds__(1024) void rank_pairs_kernel(const SetView *__restrict__ views,
                                                          const PairTask *__restrict__ tasks,
                                                          TaskQueues q, double delta) {
  __shared__ RankShared sh;
  __shared__ uint32_t s_task;
  const uint32_t tid = threadIdx.x;
  for (uint32_t x = tid; x < (uint32_t)kLogEntries; x += 1024) log_table_entry((int)x, sh.logt[x]);
  if (tid == 0) sh.ln2 = log(2.0);
  clear_rows(sh.row);
  // XCC_ID: bits 3:0 of hardware register 20
  const uint32_t home = (uint32_t)__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) % kXcdQueues;
  uint32_t empty = 0;
  for (;;) {
    if (tid == 0) s_task = take_task(q, home, empty);
    __syncthreads();
    const uint32_t t = s_task;
    __syncthreads();
    if (t == kNoTask) break;
    const PairTask tk = tasks[t];
    run_pair_task(views[tk.set], tk, sh, delta);
  }
}

hipError_t launch_rank_pairs(hipStream_t st, const SetView *d_views, const PairTask *tasks,
                             uint32_t ntasks, const TaskQueues &q, uint32_t workgroups, double delta) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_pairs_kernel, dim3(min(workgroups, ntasks)), dim3(1024), 0, st, d_views,
                     tasks, q, delta);
  return hipGetLastError();
}

// R = (sum of the pair terms + the j = i term) / N for every sorted
// position of every set; written at the sequence's input index.
__global__ void rank_finalize_kernel(Segs sg, uint32_t N, double delta, double *__restrict__ ranks,
                                     uint32_t *__restrict__ qhead) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kXcdQueues) qhead[p] = 0;  // the rank launch's queues, for the next one
  if (p >= N) return;
  const uint32_t set = sg.set_of_pos(p);
  const uint32_t a = sg.seq[set], n = sg.seq[set + 1] - a;
  const SetView &v = sg.views[set];
  long long *acc = v.acc + (p - a);
  const int fix = fix_bits(n, delta);
  const long long self = fix_q(-log(delta + 1.0), fix);  // the j = i term: F = 1
  ranks[a + v.perm[p - a]] = fix_value(*acc + self, fix) / (double)n;
  *acc = 0;  // cleared for the next rank launch
}

hipError_t launch_rank_finalize(hipStream_t st, const Segs &sg, uint32_t N, double delta,
                                double *ranks, uint32_t *qhead) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_finalize_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sg, N, delta,
                     ranks, qhead);
  return hipGetLastError();
}

// Explicit shared counts for rows rowpos[...] x columns colpos[...] (sorted
// positions).  Grid: x = row block of 16 listed rows, y = 1024 listed
// columns (16 waves x 64 lanes).
__global__ __launch_bounds__(1024) void similarity_kernel(
    SetView v, const uint32_t *__restrict__ rowpos, uint32_t nr, const uint32_t *__restrict__ colpos,
    uint32_t nc, const uint32_t *__restrict__ exc_off, const uint32_t *__restrict__ exc_n,
    const uint16_t *__restrict__ exc_ids, const uint16_t *__restrict__ exc_cnt,
    uint16_t *__restrict__ shared, uint16_t *__restrict__ denom) {
  __shared__ RowShared sh;
  const uint32_t bx = blockIdx.x;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t e0 = exc_off[bx], en = exc_n[bx];
  clear_rows(sh);
  __syncthreads();
  touch_rows<true>(v, ListedRows{rowpos + 16u * bx}, exc_ids, e0, en, sh);
  __syncthreads();
  const uint16_t *T16 = reinterpret_cast<const uint16_t *>(sh.T32);
  const uint32_t c = blockIdx.y * 1024u + wave * 64u + lane;
  const bool vc = c < nc;
  const uint32_t sc = vc ? colpos[c] : 0u;
  const uint32_t g = sc >> 6, ln = sc & 63u;
  const uint32_t L = vc ? v.grp_len[g] : 0u;
  uint32_t Lw = L;
#pragma unroll
  for (int o = 32; o; o >>= 1) Lw = max(Lw, (uint32_t)__shfl_xor((int)Lw, o, 64));
  if (Lw == 0) return;
  const uint4 *p = reinterpret_cast<const uint4 *>(v.gids + v.grp_off[g]) + ln;
  uint32_t cnt[16];
  switch (np_bucket(Lw)) {
    case 8: column_counts_ragged<8>(T16, p, L, Lw, cnt); break;
    case 10: column_counts_ragged<10>(T16, p, L, Lw, cnt); break;
    case 12: column_counts_ragged<12>(T16, p, L, Lw, cnt); break;
    case 14: column_counts_ragged<14>(T16, p, L, Lw, cnt); break;
    default: column_counts_ragged<16>(T16, p, L, Lw, cnt); break;
  }
  if (!vc) return;
  column_excess(v, sc, sh.BM, sh.BP, exc_cnt, e0, cnt);
  const uint32_t Kc = v.K[sc];
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const uint32_t row = 16u * bx + r;
    if (row < nr) {
      shared[(size_t)row * nc + c] = (uint16_t)cnt[r];
      if (denom) denom[(size_t)row * nc + c] = (uint16_t)min(sh.rowK[r], Kc);
    }
  }
}

hipError_t launch_similarity(hipStream_t st, const SetView &v, const uint32_t *rowpos, uint32_t nr,
                             const uint32_t *colpos, uint32_t nc, const uint32_t *exc_off,
                             const uint32_t *exc_n, const uint16_t *exc_ids,
                             const uint16_t *exc_cnt, uint16_t *shared, uint16_t *denom) {
  if (nr == 0 || nc == 0) return hipSuccess;
  dim3 grid((nr + 15) / 16, (nc + 1023) / 1024);
  hipLaunchKernelGGL(similarity_kernel, grid, dim3(1024), 0, st, v, rowpos, nr, colpos, nc,
                     exc_off, exc_n, exc_ids, exc_cnt, shared, denom);
  return hipGetLastError();
}

}  // namespace kd
