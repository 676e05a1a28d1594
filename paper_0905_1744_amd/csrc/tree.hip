// After the split: each bucket's sequences are gathered together (the
// redistribution of Section 3.1.2, Algorithm 2 step 11, done on one
// device), their pairwise k-mer distances form one matrix per bucket
// (Equations 1-2 for every pair of the bucket), and each matrix gives a
// UPGMA guide tree -- the similarity matrix and guide tree of the generic
// alignment scheme the paper's local alignment stage runs (Section 2,
// Section 3.1.3).
#include "radix.h"
#include "tile.h"

namespace kd {

// ------------------------------------------------------ redistribution

// length of sequence i when it is a valid entry, else 0 (and invalid)
__device__ __forceinline__ uint64_t seq_len(const uint64_t *off, uint32_t n_seqs, uint64_t nres,
                                            uint32_t i, bool &ok) {
  ok = i < n_seqs && off[i] <= off[i + 1] && off[i + 1] <= nres;
  return ok ? off[i + 1] - off[i] : 0;
}

// out_off[i] = sum of the lengths of order[0..i) (exclusive), one
// workgroup; entries of order outside [0, n_seqs), or whose offsets are
// decreasing or past nres, set *err (and count as empty).
__global__ __launch_bounds__(1024) void gather_offsets_kernel(const uint64_t *__restrict__ off,
                                                              uint32_t n_seqs, uint64_t nres,
                                                              const uint32_t *__restrict__ order,
                                                              uint32_t n, uint64_t *__restrict__ out_off,
                                                              unsigned long long *err) {
  __shared__ unsigned long long wsum[16];
  const uint32_t per = (n + 1023) / 1024;
  const uint32_t x0 = min(n, threadIdx.x * per), x1 = min(n, x0 + per);
  unsigned long long s = 0;
  bool bad = false;
  for (uint32_t x = x0; x < x1; x++) {
    bool ok;
    s += seq_len(off, n_seqs, nres, order[x], ok);
    bad |= !ok;
  }
  if (bad) atomicMin(err, 1ull);
  unsigned long long tot;
  unsigned long long run = block_exclusive_scan64<1024>(s, wsum, tot);
  for (uint32_t x = x0; x < x1; x++) {
    out_off[x] = run;
    bool ok;
    run += seq_len(off, n_seqs, nres, order[x], ok);
  }
  if (threadIdx.x == 0) out_off[n] = tot;
}

// one wave per sequence: bytes of sequence order[x] to out + out_off[x]
__global__ __launch_bounds__(256) void gather_copy_kernel(const uint8_t *__restrict__ res,
                                                          const uint64_t *__restrict__ off,
                                                          uint32_t n_seqs, uint64_t nres,
                                                          const uint32_t *__restrict__ order, uint32_t n,
                                                          const uint64_t *__restrict__ out_off,
                                                          uint64_t cap, uint8_t *__restrict__ out) {
  const uint32_t x = blockIdx.x * 4u + (threadIdx.x >> 6), lane = threadIdx.x & 63u;
  if (x >= n) return;
  bool ok;
  const uint32_t i = order[x];
  const uint64_t len = seq_len(off, n_seqs, nres, i, ok), o = out_off[x];
  if (!ok || o + len > cap) return;  // the host reports these errors
  const uint64_t a = off[i];
  for (uint64_t t = lane; t < len; t += 64) out[o + t] = res[a + t];
}

hipError_t launch_gather(hipStream_t st, const uint8_t *res, const uint64_t *off, uint32_t n_seqs,
                         uint64_t nres, const uint32_t *order, uint32_t n, uint8_t *out, uint64_t cap,
                         uint64_t *out_off, unsigned long long *err) {
  hipLaunchKernelGGL(gather_offsets_kernel, dim3(1), dim3(1024), 0, st, off, n_seqs, nres, order, n,
                     out_off, err);
  KD_HIP(hipGetLastError());
  if (n == 0 || !out) return hipSuccess;
  hipLaunchKernelGGL(gather_copy_kernel, dim3((n + 3) / 4), dim3(256), 0, st, res, off, n_seqs, nres,
                     order, n, out_off, cap, out);
  return hipGetLastError();
}

// ---------------------------------------------------- distance matrices

struct DistShared {
  RowShared row;
  LogEntry logt[kLogEntries];
  double ln2;
  alignas(16) uint16_t exc_c[kExcLds * 16];
};

// Row stride of a set's sorted-order scratch matrix: whole 128-byte lines.
__host__ __device__ inline uint64_t dist_ld(uint64_t n) { return (n + 15) & ~(uint64_t)15; }

// d for the pairs of one 16 x 64 tile below the diagonal, written at both
// (row, column) and (column, row) of the set's scratch matrix in sorted
// order (row stride dist_ld(N)): a row's 64 columns are one line-aligned
// 512-byte store, and each lane's 16 rows fill one 128-byte line of its
// column's row.  dist_permute_kernel puts them in input order.
__device__ __forceinline__ void dist_tile(const SetView &v, DistShared &sh, uint32_t rb, uint32_t g,
                                          double delta, const uint16_t *ecnt, double *__restrict__ M) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t L = __builtin_amdgcn_readfirstlane(v.grp_len[g]);
  const uint32_t hl = __builtin_amdgcn_readfirstlane(v.ghi_len[g]);
  const uint32_t sc = 64u * g + lane;
  const bool vc = sc < v.N;
  const uint4 *p = reinterpret_cast<const uint4 *>(v.gids + v.grp_off[g]) + lane;
  const uint32_t *hp = v.ghi + v.ghi_off[g] + lane;
  uint32_t q0[4] = {0u, 0u, 0u, 0u};
  if (hl > 0) {
#pragma unroll
    for (int k = 0; k < 4; k++) q0[k] = hp[(size_t)k * 64];
  }
  uint32_t cnt[16];
  column_counts(reinterpret_cast<const uint16_t *>(sh.row.T32), p, L, cnt);
  column_excess_grouped(hp, hl, q0, sh.row.BM, sh.row.BP, ecnt, cnt);
  if (!vc) return;
  const uint32_t Kc = v.K[sc];
  const double invKc = v.invK[sc];
  const uint64_t ld = dist_ld(v.N);
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const uint32_t sr = 16u * rb + r;
    if (sc < sr && sr < v.N) {
      const double inv = sh.row.rowK[r] < Kc ? sh.row.rowInv[r] : invKc;
      const double d = log_tab<true>(fma((double)cnt[r], inv, delta), sh.logt, sh.ln2);
      M[sr * ld + sc] = d;
      M[(uint64_t)sc * ld + sr] = d;
    }
  }
}

// The rank kernel's work list (strips of 32 column groups against runs of
// row blocks, pairs below the diagonal only), with the pair terms stored
// instead of summed.  soff[set] = first element of the set's scratch matrix.
__global__ __launch_bounds__(1024) void dist_pairs_kernel(const SetView *__restrict__ views,
                                                          const PairTask *__restrict__ tasks,
                                                          const uint64_t *__restrict__ soff,
                                                          double delta, double *__restrict__ scratch) {
  __shared__ DistShared sh;
  const PairTask tk = tasks[blockIdx.x];
  const SetView &v = views[tk.set];
  double *M = scratch + soff[tk.set];
  const uint32_t tid = threadIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (uint32_t q = tid; q < (uint32_t)kLogEntries; q += 1024) log_table_entry((int)q, sh.logt[q]);
  if (tid == 0) sh.ln2 = log(2.0);
  clear_rows(sh.row);
  const uint32_t ga = tk.g0 + wave, gb = tk.g0 + 31u - wave;
  for (uint32_t rb = tk.rb0; rb < tk.rb1; rb++) {
    if (rb > tk.rb0) {
      const uint32_t pr = rb - 1;
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
    if (ga < v.G && rb >= 4u * ga) dist_tile(v, sh, rb, ga, delta, ecnt, M);
    if (gb < v.G && rb >= 4u * gb) dist_tile(v, sh, rb, gb, delta, ecnt, M);
    __syncthreads();
  }
}

// Input order: row r of a set's matrix is row inv[r] of its scratch matrix
// with the columns permuted, M[r][c] = scratch[inv[r]][inv[c]]; the
// diagonal (F(i, i) = 1) is d = -ln(delta + 1).  One workgroup per row: the
// scratch row is read whole (coalesced) into LDS, the matrix row written
// whole.  ROWS_IN_LDS false (sets beyond the LDS): the columns are read from
// the scratch row in memory.
template <bool ROWS_IN_LDS>
__global__ __launch_bounds__(256) void dist_permute_kernel(Segs sg, const SetView *__restrict__ views,
                                                           const uint64_t *__restrict__ soff,
                                                           const uint64_t *__restrict__ doff, double delta,
                                                           const double *__restrict__ scratch,
                                                           double *__restrict__ dist) {
  extern __shared__ double row[];
  const uint32_t p = blockIdx.x;
  const uint32_t set = sg.set_of_pos(p);
  const SetView &v = views[set];
  const uint32_t n = v.N, r = p - v.base;
  const double *src = scratch + soff[set] + (uint64_t)v.inv[r] * dist_ld(n);
  if (ROWS_IN_LDS) {
    for (uint32_t c = threadIdx.x; c < n; c += 256) row[c] = src[c];
    __syncthreads();
  }
  const double diag = -log(delta + 1.0);
  double *dst = dist + doff[set] + (uint64_t)r * n;
  for (uint32_t c = threadIdx.x; c < n; c += 256) {
    const uint32_t sc = v.inv[c];
    dst[c] = c == r ? diag : (ROWS_IN_LDS ? row[sc] : src[sc]);
  }
}

hipError_t launch_distances(hipStream_t st, const Segs &sg, uint32_t N, uint32_t max_n, const SetView *d_views,
                            const PairTask *tasks, uint32_t ntasks, const uint64_t *soff, const uint64_t *doff,
                            double delta, double *scratch, double *dist) {
  if (N == 0) return hipSuccess;
  if (ntasks) {
    hipLaunchKernelGGL(dist_pairs_kernel, dim3(ntasks), dim3(1024), 0, st, d_views, tasks, soff, delta,
                       scratch);
    KD_HIP(hipGetLastError());
  }
  if (max_n <= kDistLdsRow)
    hipLaunchKernelGGL(dist_permute_kernel<true>, dim3(N), dim3(256), sizeof(double) * max_n, st, sg, d_views,
                       soff, doff, delta, scratch, dist);
  else
    hipLaunchKernelGGL(dist_permute_kernel<false>, dim3(N), dim3(256), 0, st, sg, d_views, soff, doff, delta,
                       scratch, dist);
  return hipGetLastError();
}

// ------------------------------------------------------------------ UPGMA
//
// One workgroup per set, on a full symmetric copy D of its matrix (n x n,
// n <= kTreeMax).  The slot rule, tie rule and update arithmetic are those
// of the definition (merge the active slots a < b with the smallest
// D[a][b], ties to the smallest a then b; the merged cluster keeps slot a;
// D[a][k] = (n_a D[a][k] + n_b D[b][k]) / (n_a + n_b) rounded step by step
// in double), so the same matrix gives the same merges and heights.
//
// To find the pair, row k keeps the minimum of D[k][j] over active j > k
// and its smallest argument.  After merging a and b: row a is recomputed
// while its entries are updated; a row k < a takes the new D[k][a] if it
// is smaller (or equal with a smaller column); rows k < b whose minimum sat
// at column a or b are rescanned, reading the old row with columns a and b
// left out (the new D[k][a] is added to the result).
//
// Waves 0-7 own the rows (thread tid: rows tid, tid + 512, ...; only the
// owner keeps a row's minimum); waves 8-15 rescan.  A merge has two
// barriers.  Before the first, each owner wave reduces the pair itself,
// loads its rows' entries of rows a and b, and lists its rows that need a
// rescan; after it the rescanning waves take the listed rows (8 / rows
// waves per row) while the owners store the new entries, and all leave
// partial minima in LDS: row a's, the next pair's over the owners' other
// rows, and the rescans' parts, all keyed by (minimum, row << 16 |
// argument) so that the argument travels with the row.  After the second
// barrier the owners reduce them to the next pair and take their rows'
// new minima from them.

constexpr uint32_t kTreeMax = kTreeMaxSeqs;
constexpr uint16_t kNone16 = 0xFFFFu;
constexpr int kTreeWaves = 16;  // waves of the merge kernel
constexpr int kTreeRowWaves = 8;  // of which own rows (the rest rescan)

// a row's state in one 16-byte record: one address per row, the fields at
// immediate offsets
struct TreeRow {
  double min;     // minimum of the row's entries right of the diagonal
  uint16_t arg;   // its smallest column (kNone16: no entry)
  uint16_t size;  // the cluster's size and id
  uint16_t id;
  uint16_t pad;
};

struct TreeShared {
  TreeRow row[kTreeMax];
  uint32_t act[kTreeMax / 32];  // bit k: slot k still in use
  uint16_t redo[kTreeMax];   // rows rescanned in this merge
  double partv[kTreeMax];    // the rescans' keyed parts
  uint32_t parti[kTreeMax];
  // wave partials, two buffers by merge parity: the next pair, row a
  double pv[2][16], av[2][16];
  uint32_t pi[2][16], ai[2][16];
  uint32_t nredo[2];         // by merge parity
  uint32_t cur[2];           // the pair (a, b), for the rescanning waves
  uint32_t stop;             // no comparable pair left
};

__device__ __forceinline__ bool slot_active(const uint32_t *act, uint32_t j) {
  return (act[j >> 5] >> (j & 31u)) & 1u;
}
struct BitActive {
  const uint32_t *act;
  __device__ bool operator()(uint32_t j) const { return slot_active(act, j); }
};

// lexicographic (value, index) minimum
__device__ __forceinline__ void lex_min(double &v, uint32_t &i, double v2, uint32_t i2) {
  const bool take = (v2 < v) | ((v2 == v) & (i2 < i));  // no short circuit: selects, not branches
  v = take ? v2 : v;
  i = take ? i2 : i;
}

// The wave reductions below find the smallest value first (v_min_f64, two
// moves and a minimum per step), then the smallest index among the lanes
// holding it (one move and a minimum per step): half the instructions of
// carrying (value, index) pairs through every step.  Neither is ever NaN
// here (lex_min never takes a NaN), so the value found is some lane's
// value; the result's value is read from the winning lane (so that a zero
// keeps the sign of the winner's).

// the lane that the DPP control CTRL names, in the rows of ROWS (other
// rows read their own value)
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_fmin(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  return __builtin_fmin(v, __hiloint2double(hi2, lo2));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_umin(uint32_t i) {
  const uint32_t i2 = (uint32_t)__builtin_amdgcn_update_dpp((int)i, (int)i, CTRL, ROWS, 0xF, false);
  return i < i2 ? i : i2;
}

__device__ __forceinline__ double read_lane(double v, uint32_t l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// the index pass and the winner's value, given the value minimum m (uniform)
__device__ __forceinline__ void lex_finish(double &v, uint32_t &i, double m, uint32_t j,
                                           unsigned long long lanes) {
  const unsigned long long w = __ballot(v == m && i == j) & lanes;
  v = w ? read_lane(v, (uint32_t)__builtin_ctzll(w)) : m;
  i = j;
}

// lexicographic (value, index) minimum over lanes 0-15, returned in every
// lane: quad swaps (1 0 3 2, 2 3 0 1), then the half-row and row mirrors
__device__ __forceinline__ void row_lex_min(double &v, uint32_t &i) {
  double m = dpp_fmin<0xB1, 0xF>(v);  // quad_perm 1 0 3 2
  m = dpp_fmin<0x4E, 0xF>(m);         // quad_perm 2 3 0 1
  m = dpp_fmin<0x141, 0xF>(m);        // row_half_mirror
  m = dpp_fmin<0x140, 0xF>(m);        // row_mirror
  m = read_lane(m, 0);
  uint32_t j = v == m ? i : 0xFFFFFFFFu;
  j = dpp_umin<0xB1, 0xF>(j);
  j = dpp_umin<0x4E, 0xF>(j);
  j = dpp_umin<0x141, 0xF>(j);
  j = dpp_umin<0x140, 0xF>(j);
  j = (uint32_t)__builtin_amdgcn_readlane((int)j, 0);
  lex_finish(v, i, m, j, 0xFFFFull);
}

// the same over the 64 lanes (all lanes active): after the row steps, row
// 15 broadcast into rows 1 and 3, then row 31 broadcast into rows 2 and 3
// leave the wave's minimum in lane 63.  The minimum of a total order does
// not depend on the combining order.
__device__ __forceinline__ void wave_lex_min(double &v, uint32_t &i) {
  double m = dpp_fmin<0xB1, 0xF>(v);
  m = dpp_fmin<0x4E, 0xF>(m);
  m = dpp_fmin<0x141, 0xF>(m);
  m = dpp_fmin<0x140, 0xF>(m);
  m = dpp_fmin<0x142, 0xA>(m);  // row_bcast:15
  m = dpp_fmin<0x143, 0xC>(m);  // row_bcast:31
  m = read_lane(m, 63);
  uint32_t j = v == m ? i : 0xFFFFFFFFu;
  j = dpp_umin<0xB1, 0xF>(j);
  j = dpp_umin<0x4E, 0xF>(j);
  j = dpp_umin<0x141, 0xF>(j);
  j = dpp_umin<0x140, 0xF>(j);
  j = dpp_umin<0x142, 0xA>(j);
  j = dpp_umin<0x143, 0xC>(j);
  j = (uint32_t)__builtin_amdgcn_readlane((int)j, 63);
  lex_finish(v, i, m, j, ~0ull);
}

// Minimum of D[k][j] over active columns j > k other than s1 and s2, with
// its smallest argument, in every lane (U loads in flight per lane).
template <int U = 8, class Active>
__device__ __forceinline__ void row_min(const double *D, uint32_t n, uint32_t k, uint32_t s1, uint32_t s2,
                                        Active active, double &v, uint32_t &i) {
  const uint32_t lane = threadIdx.x & 63u;
  v = __builtin_inf();
  i = 0xFFFFFFFFu;
  const char *row = reinterpret_cast<const char *>(D + (size_t)k * n);  // k uniform: a scalar base
  for (uint32_t j0 = k + 1; j0 < n; j0 += 64u * U) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; u++) {  // clamped, not branched: every load goes out at once
      const uint32_t j = min(j0 + 64u * u + lane, n - 1);
      x[u] = *reinterpret_cast<const double *>(row + 8u * j);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t j = j0 + 64u * u + lane;
      if (j < n && j != s1 && j != s2 && active(j)) lex_min(v, i, x[u], j);
    }
  }
  wave_lex_min(v, i);
}

struct AllActive {
  __device__ bool operator()(uint32_t) const { return true; }
};

#pragma clang fp contract(off)
__device__ __forceinline__ double merge_mean(double na, double x, double nb, double y) {
  const double p = na * x;
  const double q = nb * y;
  const double s = p + q;
  return s / (na + nb);
}

// Initial row minima of every set, one wave per row, all sets at once.
__global__ __launch_bounds__(256) void upgma_init_kernel(const uint32_t *__restrict__ first,
                                                         uint32_t nsets,
                                                         const uint64_t *__restrict__ doff,
                                                         const double *__restrict__ work,
                                                         double *__restrict__ rmin,
                                                         uint32_t *__restrict__ rarg) {
  const uint32_t p = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (p >= first[nsets]) return;
  uint32_t lo = 0, hi = nsets;  // set of row p: last set with first[set] <= p
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (first[mid] <= p) lo = mid;
    else hi = mid;
  }
  const uint32_t n = first[lo + 1] - first[lo], k = p - first[lo];
  double v;
  uint32_t i;
  row_min(work + doff[lo], n, k, 0xFFFFFFFFu, 0xFFFFFFFFu, AllActive{}, v, i);
  if ((threadIdx.x & 63u) == 0) {
    rmin[p] = v;
    rarg[p] = i;
  }
}

// pair key of row k: its minimum's argument (kNone16 when it has none) in
// the low half, the row above it
__device__ __forceinline__ uint32_t pair_key(uint32_t k, uint32_t arg) {
  return (k << 16) | (arg < kNone16 ? arg : kNone16);
}

// A set whose remaining pairs compare false with everything (NaN
// distances) stops there and records its index in *err.
//
// Waves 0 .. RW-1 own the rows (thread tid: rows tid, tid + 64 RW, ...;
// PER of them); the other waves only rescan.
template <int RW, int PER>
__global__ __launch_bounds__(64 * kTreeWaves) void upgma_kernel(const uint32_t *__restrict__ first,
                                                                const uint64_t *__restrict__ doff,
                                                                double *__restrict__ work,
                                                                const double *__restrict__ rmin,
                                                                const uint32_t *__restrict__ rarg,
                                                                int32_t *__restrict__ merges,
                                                                double *__restrict__ heights,
                                                                unsigned long long *err) {
  constexpr uint32_t RT = 64u * RW;  // threads that own rows
  constexpr uint32_t RS = kTreeWaves - RW;  // rescanning waves
  constexpr uint32_t kLogRS = __builtin_ctz(RS);
  static_assert((RS & (RS - 1)) == 0 && RS <= 16 && RW <= 16, "wave partials hold 16 entries");
  constexpr int kRescanLoads = 8;  // loads in flight per lane in a rescan
  constexpr uint32_t kNo = 0xFFFFFFFFu;
  __shared__ TreeShared sh;
  const uint32_t set = blockIdx.x;
  const uint32_t f0 = first[set], n = first[set + 1] - f0;
  double *D = work + doff[set];
  int32_t *mg = merges + 2ull * (f0 - set);
  double *ht = heights + (f0 - set);
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool rows = wave < RW;
  if (n < 2) return;
  // state, and the first pair's partials (buffer 0; no merged row or
  // rescans yet)
  for (uint32_t w = tid; w < kTreeMax / 32; w += 64u * kTreeWaves)
    sh.act[w] = 32 * w + 32 <= n ? ~0u : (32 * w < n ? (1u << (n - 32 * w)) - 1u : 0u);
  if (rows) {
    double v = __builtin_inf();
    uint32_t i = kNo;
    for (uint32_t k = tid; k < n; k += RT) {
      const double m = rmin[f0 + k];
      const uint32_t r = rarg[f0 + k];
      sh.row[k].size = 1;
      sh.row[k].id = (uint16_t)k;
      sh.row[k].min = m;
      sh.row[k].arg = r < kNone16 ? (uint16_t)r : kNone16;
      lex_min(v, i, m, pair_key(k, r));
    }
    wave_lex_min(v, i);
    if (lane == 0) {
      sh.pv[0][wave] = v;
      sh.pi[0][wave] = i;
    }
    if (tid == 0) sh.nredo[0] = sh.nredo[1] = 0;
  }
  __syncthreads();
  uint32_t pa = kNo, pb = kNo;  // the previous merge's slots
  double npa = 0.0;             // and the merged cluster's size
  uint32_t np = 0, pw = 1;      // its rescans: parts, parts per row
  // this thread's rows rescanned in the previous merge (bit u) and their
  // places in the list (the entry a row adds to its rescan waits in its
  // own minimum's slot)
  uint32_t redo = 0;
  uint32_t qpos[PER];
#pragma unroll
  for (int u = 0; u < PER; u++) qpos[u] = 0;
  for (uint32_t t = 0; t + 1 < n; t++) {
    const uint32_t buf = t & 1u;
    uint32_t a = 0, b = 0;
    double na = 1.0, nb = 1.0, h = 0.0;
    double xa[PER], xb[PER], rm[PER];  // the rows' values, from one barrier to the next
    uint32_t ra[PER];
    bool use[PER];
    if (rows) {
      // the pair: the wave partials over the rows other than pa, row pa's
      // partials and the rescans' parts (each keyed as its row)
      double v = __builtin_inf();
      uint32_t i = kNo;
      if (lane < RW) {
        v = sh.pv[buf][lane];
        i = sh.pi[buf][lane];
        if (pa != kNo) lex_min(v, i, sh.av[buf][lane], pair_key(pa, sh.ai[buf][lane]));
      }
      for (uint32_t p = lane; p < np; p += 64) lex_min(v, i, sh.partv[p], sh.parti[p]);
      if (np <= 16) row_lex_min(v, i);  // everything in lanes 0-15
      else wave_lex_min(v, i);
      h = v;
      a = i >> 16;
      b = i & 0xFFFFu;
      const bool bad = a >= n || b >= n;
      if (tid == 0) {
        sh.cur[0] = a;
        sh.cur[1] = b;
        sh.stop = bad;
      }
      if (!bad) {
        // this thread's entries of rows a and b, out first
#pragma unroll
        for (int u = 0; u < PER; u++) {
          const uint32_t k = tid + RT * u;
          xa[u] = k < n ? D[(size_t)a * n + k] : 0.0;
          xb[u] = k < n ? D[(size_t)b * n + k] : 0.0;
        }
        if (pa != kNo) {
          // the previous merge's bookkeeping: row pa's minimum and the
          // rescanned rows' minima (their owners keep them), slot pb
          // retired, the merged cluster's size and id, the previous
          // rescan count cleared
          if (wave == (pa % RT) >> 6) {
            double va = lane < RW ? sh.av[buf][lane] : __builtin_inf();
            uint32_t ia = lane < RW ? sh.ai[buf][lane] : kNo;
            row_lex_min(va, ia);
            if (lane == pa % 64u) {
              sh.row[pa].min = va;
              sh.row[pa].arg = ia < kNone16 ? (uint16_t)ia : kNone16;
            }
          }
#pragma unroll
          for (int u = 0; u < PER; u++) {
            if (!((redo >> u) & 1u)) continue;
            const uint32_t k = tid + RT * u;
            double rv = sh.row[k].min;
            uint32_t ri = pair_key(k, sh.row[k].arg);
            for (uint32_t p = qpos[u] * pw; p < (qpos[u] + 1) * pw; p++) lex_min(rv, ri, sh.partv[p], sh.parti[p]);
            sh.row[k].min = rv;
            sh.row[k].arg = (uint16_t)(ri & 0xFFFFu);
          }
          if (tid == pb % RT) atomicAnd(&sh.act[pb >> 5], ~(1u << (pb & 31u)));
          if (tid == 0) {
            sh.row[pa].size = (uint16_t)npa;
            sh.row[pa].id = (uint16_t)(n + t - 1);
            sh.nredo[buf ^ 1u] = 0;
          }
        }
        // this thread's rows' minima, and the rows that need a rescan listed
        redo = 0;
#pragma unroll
        for (int u = 0; u < PER; u++) {
          const uint32_t k = tid + RT * u;
          use[u] = k < n && slot_active(sh.act, k) && k != a && k != b;
          rm[u] = use[u] ? sh.row[k].min : 0.0;
          ra[u] = use[u] ? sh.row[k].arg : kNone16;
          if (use[u] && (k < a ? (ra[u] == a || ra[u] == b) : (k < b && ra[u] == b))) {
            redo |= 1u << u;
            qpos[u] = atomicAdd(&sh.nredo[buf], 1u);
            sh.redo[qpos[u]] = (uint16_t)k;
          }
        }
      }
    }
    __syncthreads();  // the pair and the rescan list are complete
    if (sh.stop) {
      if (tid == 0) atomicMin(err, (unsigned long long)set);
      return;
    }
    const uint32_t nr = sh.nredo[buf];
    if (rows) {
      na = a == pa ? npa : (double)sh.row[a].size;
      nb = b == pa ? npa : (double)sh.row[b].size;
      if (tid == 0) {
        const int32_t x = a == pa ? (int32_t)(n + t - 1) : sh.row[a].id;
        const int32_t y = b == pa ? (int32_t)(n + t - 1) : sh.row[b].id;
        mg[2 * t] = x < y ? x : y;
        mg[2 * t + 1] = x < y ? y : x;
        ht[t] = h / 2.0;
      }
      // the merged row's entries; row a's minimum, and the next pair's over
      // the other rows not rescanned (a rescanned row k < a adds its new
      // entry at column a)
      double av = __builtin_inf(), pv = __builtin_inf();
      uint32_t ai = kNo, pi = kNo;
#pragma unroll
      for (int u = 0; u < PER; u++) {
        const uint32_t k = tid + RT * u;
        if (!use[u]) continue;
        const double nv = merge_mean(na, xa[u], nb, xb[u]);
        D[(size_t)a * n + k] = nv;
        D[(size_t)k * n + a] = nv;
        if (k > a) lex_min(av, ai, nv, k);
        if ((redo >> u) & 1u) {
          const double cv = k < a ? nv : __builtin_inf();
          const uint32_t ca = k < a ? a : kNone16;
          sh.row[k].min = cv;
          sh.row[k].arg = (uint16_t)ca;
          lex_min(pv, pi, cv, pair_key(k, ca));
          continue;
        }
        if (k < a) {
          if (nv < rm[u] || (nv == rm[u] && a < ra[u])) {
            rm[u] = nv;
            ra[u] = a;
          }
          sh.row[k].min = rm[u];
          sh.row[k].arg = (uint16_t)ra[u];
        }
        lex_min(pv, pi, rm[u], pair_key(k, ra[u]));
      }
      wave_lex_min(av, ai);
      wave_lex_min(pv, pi);
      if (lane == 0) {
        sh.av[buf ^ 1u][wave] = av;
        sh.ai[buf ^ 1u][wave] = ai;
        sh.pv[buf ^ 1u][wave] = pv;
        sh.pi[buf ^ 1u][wave] = pi;
      }
    } else if (nr > 0) {
      // the rescans, of the old rows without columns a and b: up to RS
      // rows, W waves per row (RS / rows rounded down to a power of two),
      // else whole rows in turn
      a = sh.cur[0];
      b = sh.cur[1];
      const uint32_t rw = wave - RW;
      if (nr <= RS) {
        const uint32_t lw = nr == 1 ? kLogRS : kLogRS - (32u - __builtin_clz(nr - 1));
        const uint32_t W = 1u << lw, q = rw >> lw, part = rw & (W - 1u);
        if (q < nr) {
          const uint32_t rk = sh.redo[q];
          const char *rrow = reinterpret_cast<const char *>(D + (size_t)rk * n);
          double v2 = __builtin_inf();
          uint32_t i2 = kNo;
          for (uint32_t j0 = rk + 1 + 64u * part; j0 < n; j0 += 64u * W * kRescanLoads) {
            double rx[kRescanLoads];
#pragma unroll
            for (int u = 0; u < kRescanLoads; u++) {
              const uint32_t j = min(j0 + 64u * W * u + lane, n - 1);
              rx[u] = *reinterpret_cast<const double *>(rrow + 8u * j);
            }
#pragma unroll
            for (int u = 0; u < kRescanLoads; u++) {
              const uint32_t j = j0 + 64u * W * u + lane;
              if (j < n && j != a && j != b && slot_active(sh.act, j)) lex_min(v2, i2, rx[u], j);
            }
          }
          wave_lex_min(v2, i2);
          if (lane == 0) {
            sh.partv[rw] = v2;
            sh.parti[rw] = pair_key(rk, i2);
          }
        }
      } else {
        for (uint32_t q = rw; q < nr; q += RS) {
          const uint32_t k = sh.redo[q];
          double v2;
          uint32_t i2;
          row_min<kRescanLoads>(D, n, k, a, b, BitActive{sh.act}, v2, i2);
          if (lane == 0) {
            sh.partv[q] = v2;
            sh.parti[q] = pair_key(k, i2);
          }
        }
      }
    }
    __syncthreads();  // D, the rows' minima, the partials and the parts are complete
    const uint32_t lw = nr <= 1 ? kLogRS : (nr <= RS ? kLogRS - (32u - __builtin_clz(nr - 1)) : 0u);
    pw = nr > 0 && nr <= RS ? (1u << lw) : 1u;
    np = nr > 0 && nr <= RS ? nr << lw : nr;
    pa = a;
    pb = b;
    npa = na + nb;
  }
}

hipError_t launch_upgma(hipStream_t st, uint32_t nsets, uint32_t N, uint32_t max_n, const uint32_t *first,
                        const uint64_t *doff, double *work, double *rmin, uint32_t *rarg,
                        int32_t *merges, double *heights, unsigned long long *err) {
  if (nsets == 0 || N == 0) return hipSuccess;
  if (max_n > kTreeMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(upgma_init_kernel, dim3((N + 3) / 4), dim3(256), 0, st, first, nsets, doff, work,
                     rmin, rarg);
  KD_HIP(hipGetLastError());
  // rows per owner thread sized to the largest set (registers for the
  // most rows only where needed)
  constexpr uint32_t RT = 64u * kTreeRowWaves;
  const dim3 grid(nsets), block(64 * kTreeWaves);
  if (max_n <= 2 * RT)
    hipLaunchKernelGGL((upgma_kernel<kTreeRowWaves, 2>), grid, block, 0, st, first, doff, work, rmin, rarg,
                       merges, heights, err);
  else if (max_n <= 4 * RT)
    hipLaunchKernelGGL((upgma_kernel<kTreeRowWaves, 4>), grid, block, 0, st, first, doff, work, rmin, rarg, merges,
                       heights, err);
  else
    hipLaunchKernelGGL((upgma_kernel<kTreeRowWaves, (kTreeMax + RT - 1) / RT>),
                       grid, block, 0, st, first, doff, work, rmin, rarg, merges, heights, err);
  return hipGetLastError();
}

}  // namespace kd
