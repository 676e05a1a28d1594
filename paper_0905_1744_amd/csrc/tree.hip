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
// at column a or b are rescanned (one wave per row).

constexpr uint32_t kTreeMax = kTreeMaxSeqs;
constexpr uint16_t kNone16 = 0xFFFFu;

struct TreeShared {
  double rowmin[kTreeMax];
  uint16_t rowarg[kTreeMax];
  uint16_t size[kTreeMax];
  uint16_t id[kTreeMax];
  uint16_t redo[kTreeMax];
  uint8_t act[kTreeMax];
  double wv[16], wv2[16];  // wave results: the pair, row a's new minimum
  uint32_t wi[16], wi2[16];
  uint32_t nredo;
  uint32_t best_a;
};

// lexicographic (value, index) minimum
__device__ __forceinline__ void lex_min(double &v, uint32_t &i, double v2, uint32_t i2) {
  const bool take = (v2 < v) | ((v2 == v) & (i2 < i));  // no short circuit: selects, not branches
  v = take ? v2 : v;
  i = take ? i2 : i;
}

// one step of the wave reduction: combine with the lane that the DPP control
// CTRL names, in the rows of ROWS (other rows keep their value)
template <int CTRL, int ROWS>
__device__ __forceinline__ void dpp_lex_step(double &v, uint32_t &i) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  const int i2 = __builtin_amdgcn_update_dpp((int)i, (int)i, CTRL, ROWS, 0xF, false);
  lex_min(v, i, __hiloint2double(hi2, lo2), (uint32_t)i2);
}

// lexicographic (value, index) minimum over the 64 lanes, in every lane
// (all lanes active).  Register-to-register moves instead of LDS permutes:
// quad swaps (1 0 3 2, 2 3 0 1), then the half-row and row mirrors leave
// each 16-lane row's minimum in all its lanes; row 15 broadcast into rows 1
// and 3 and row 31 broadcast into rows 2 and 3 leave the wave's in lane 63.
// The minimum of a total order does not depend on the combining order.
__device__ __forceinline__ void wave_lex_min(double &v, uint32_t &i) {
  dpp_lex_step<0xB1, 0xF>(v, i);   // quad_perm 1 0 3 2
  dpp_lex_step<0x4E, 0xF>(v, i);   // quad_perm 2 3 0 1
  dpp_lex_step<0x141, 0xF>(v, i);  // row_half_mirror
  dpp_lex_step<0x140, 0xF>(v, i);  // row_mirror
  dpp_lex_step<0x142, 0xA>(v, i);  // row_bcast:15
  dpp_lex_step<0x143, 0xC>(v, i);  // row_bcast:31
  v = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                       __builtin_amdgcn_readlane(__double2loint(v), 63));
  i = (uint32_t)__builtin_amdgcn_readlane((int)i, 63);
}

// Minimum of D[k][j] over columns j > k that are active and not `skip`,
// with its smallest argument, over the columns of part p of W parts (one
// wave per part, eight loads in flight per lane; W = 1: the whole row).
template <class Active>
__device__ __forceinline__ void row_min(const double *D, uint32_t n, uint32_t k, uint32_t skip,
                                        Active active, double &v, uint32_t &i, uint32_t p = 0,
                                        uint32_t W = 1) {
  const uint32_t lane = threadIdx.x & 63u;
  v = __builtin_inf();
  i = 0xFFFFFFFFu;
  const double *row = D + (size_t)k * n;
  const uint32_t stride = 64u * W;
  for (uint32_t j0 = k + 1 + 64u * p; j0 < n; j0 += 8u * stride) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const uint32_t j = j0 + stride * u + lane;
      x[u] = j < n ? row[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const uint32_t j = j0 + stride * u + lane;
      if (j < n && j != skip && active(j)) lex_min(v, i, x[u], j);
    }
  }
  wave_lex_min(v, i);
}

struct AllActive {
  __device__ bool operator()(uint32_t) const { return true; }
};
struct LdsActive {
  const uint8_t *act;
  __device__ bool operator()(uint32_t j) const { return act[j] != 0; }
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
  row_min(work + doff[lo], n, k, 0xFFFFFFFFu, AllActive{}, v, i);
  if ((threadIdx.x & 63u) == 0) {
    rmin[p] = v;
    rarg[p] = i;
  }
}

// A set whose remaining pairs compare false with everything (NaN
// distances) stops there and records its index in *err.
__global__ __launch_bounds__(1024) void upgma_kernel(const uint32_t *__restrict__ first,
                                                     const uint64_t *__restrict__ doff,
                                                     double *__restrict__ work,
                                                     const double *__restrict__ rmin,
                                                     const uint32_t *__restrict__ rarg,
                                                     int32_t *__restrict__ merges,
                                                     double *__restrict__ heights,
                                                     unsigned long long *err) {
  __shared__ TreeShared sh;
  const uint32_t set = blockIdx.x;
  const uint32_t f0 = first[set], n = first[set + 1] - f0;
  double *D = work + doff[set];
  int32_t *mg = merges + 2ull * (f0 - set);
  double *ht = heights + (f0 - set);
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  for (uint32_t k = tid; k < n; k += 1024) {
    sh.size[k] = 1;
    sh.id[k] = (uint16_t)k;
    sh.act[k] = 1;
    sh.rowmin[k] = rmin[f0 + k];
    sh.rowarg[k] = rarg[f0 + k] == 0xFFFFFFFFu ? kNone16 : (uint16_t)rarg[f0 + k];
  }
  if (tid == 0) sh.nredo = 0;
  __syncthreads();
  for (uint32_t t = 0; t + 1 < n; t++) {
    // the pair: lexicographic minimum of (rowmin[a], a) over active a
    // (a retired row's minimum is NaN, which no comparison selects: no
    // test of act, and the rows' reads go out together); every wave
    // reduces the 16 wave results itself (no second barrier)
    constexpr int kPer = kTreeMax / 1024;
    double v = __builtin_inf();
    uint32_t i = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      const uint32_t a = tid + 1024u * u;
      if (a < n) lex_min(v, i, sh.rowmin[a], a);
    }
    wave_lex_min(v, i);
    if (lane == 0) {
      sh.wv[wave] = v;
      sh.wi[wave] = i;
    }
    __syncthreads();
    v = lane < 16 ? sh.wv[lane] : __builtin_inf();
    i = lane < 16 ? sh.wi[lane] : 0xFFFFFFFFu;
    wave_lex_min(v, i);
    const uint32_t a = i;
    if (a >= n || sh.rowarg[a] == kNone16) {
      if (tid == 0) atomicMin(err, (unsigned long long)set);
      return;
    }
    const uint32_t b = sh.rowarg[a];
    const double h = sh.rowmin[a];
    const double na = (double)sh.size[a], nb = (double)sh.size[b];
    if (tid == 0) {
      const int32_t x = sh.id[a], y = sh.id[b];
      mg[2 * t] = x < y ? x : y;
      mg[2 * t + 1] = x < y ? y : x;
      ht[t] = h / 2.0;
    }
    // update row and column a (loads first, then the arithmetic); row a's
    // new minimum; rows that must rescan
    double xa[kPer], xb[kPer];
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      const uint32_t k = tid + 1024u * u;
      const bool use = k < n && sh.act[k] && k != a && k != b;
      xa[u] = use ? D[(size_t)a * n + k] : 0.0;
      xb[u] = use ? D[(size_t)b * n + k] : 0.0;
    }
    v = __builtin_inf();
    i = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      const uint32_t k = tid + 1024u * u;
      if (!(k < n && sh.act[k] && k != a && k != b)) continue;
      const double nv = merge_mean(na, xa[u], nb, xb[u]);
      D[(size_t)a * n + k] = nv;
      D[(size_t)k * n + a] = nv;
      if (k > a) {
        lex_min(v, i, nv, k);
        if (k < b && sh.rowarg[k] == b) sh.redo[atomicAdd(&sh.nredo, 1u)] = (uint16_t)k;
      } else {
        const uint16_t ra = sh.rowarg[k];
        if (ra == a || ra == b) sh.redo[atomicAdd(&sh.nredo, 1u)] = (uint16_t)k;
        else if (nv < sh.rowmin[k] || (nv == sh.rowmin[k] && a < ra)) {
          sh.rowmin[k] = nv;
          sh.rowarg[k] = (uint16_t)a;
        }
      }
    }
    wave_lex_min(v, i);
    if (lane == 0) {  // a second buffer: slower waves may still read wv
      sh.wv2[wave] = v;
      sh.wi2[wave] = i;
    }
    __syncthreads();  // row a's parts, D and the redo list are complete
    const uint32_t nr = sh.nredo;
    if (wave == 0) {
      v = lane < 16 ? sh.wv2[lane] : __builtin_inf();
      i = lane < 16 ? sh.wi2[lane] : 0xFFFFFFFFu;
      wave_lex_min(v, i);
      if (lane == 0) {
        sh.rowmin[a] = v;
        sh.rowarg[a] = i == 0xFFFFFFFFu ? kNone16 : (uint16_t)i;
        sh.act[b] = 0;
        sh.rowmin[b] = __builtin_nan("");  // never the pair's minimum
        sh.size[a] = (uint16_t)(sh.size[a] + sh.size[b]);
        sh.id[a] = (uint16_t)(n + t);
      }
    }
    // rescans skip b explicitly (its slot is retired by wave 0 meanwhile).
    // Up to 16 rows: W = 16 / rows waves share each row and their parts
    // meet in LDS; more rows: one wave per row.
    if (nr > 0 && nr <= 16) {
      const uint32_t W = 16u / nr, q = wave / W;
      if (q < nr) {
        row_min(D, n, sh.redo[q], b, LdsActive{sh.act}, v, i, wave % W, W);
        if (lane == 0) {
          sh.wv[wave] = v;
          sh.wi[wave] = i;
        }
      }
      __syncthreads();
      if (tid < nr) {
        v = __builtin_inf();
        i = 0xFFFFFFFFu;
        for (uint32_t w = tid * W; w < (tid + 1) * W; w++) lex_min(v, i, sh.wv[w], sh.wi[w]);
        const uint32_t k = sh.redo[tid];
        sh.rowmin[k] = v;
        sh.rowarg[k] = i == 0xFFFFFFFFu ? kNone16 : (uint16_t)i;
      }
    } else {
      for (uint32_t q = wave; q < nr; q += 16) {
        const uint32_t k = sh.redo[q];
        row_min(D, n, k, b, LdsActive{sh.act}, v, i);
        if (lane == 0) {
          sh.rowmin[k] = v;
          sh.rowarg[k] = i == 0xFFFFFFFFu ? kNone16 : (uint16_t)i;
        }
      }
    }
    __syncthreads();
    if (tid == 0) sh.nredo = 0;
  }
}

hipError_t launch_upgma(hipStream_t st, uint32_t nsets, uint32_t N, const uint32_t *first,
                        const uint64_t *doff, double *work, double *rmin, uint32_t *rarg,
                        int32_t *merges, double *heights, unsigned long long *err) {
  if (nsets == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(upgma_init_kernel, dim3((N + 3) / 4), dim3(256), 0, st, first, nsets, doff, work,
                     rmin, rarg);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(upgma_kernel, dim3(nsets), dim3(1024), 0, st, first, doff, work, rmin, rarg, merges,
                     heights, err);
  return hipGetLastError();
}

}  // namespace kd
