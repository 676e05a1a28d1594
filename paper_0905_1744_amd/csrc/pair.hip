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
// adds the partial sums to the rows' and columns' accumulators as exact
// 120-bit fixed-point integers (three 40-bit limbs).  Integer addition is
// associative, so R_i (Equation 3) is independent of tiling, scheduling and
// co-running work.  Each unordered pair is computed once (column position
// below row position in the sorted order), and the j = i term is added by
// the finalize kernel.
#include "tile.h"

namespace kd {

// One workgroup = 16 waves x 2 = 32 consecutive column groups g0..g0+31
// (wave w takes g0 + w and g0 + 31 - w: lists grow with g, so every wave
// gets about the same total length) against row blocks rb0..rb1-1, one
// row block at a time.  Row partials of a row block meet in LDS (exact
// integer adds) and go to HBM once; column partials stay in registers
// across the row blocks and go to HBM once at the end.
__global__ __launch_bounds__(1024) void rank_pairs_kernel(const SetView *__restrict__ views,
                                                          const PairTask *__restrict__ tasks,
                                                          double delta) {
  __shared__ RankShared sh;
  const PairTask tk = tasks[blockIdx.x];
  const SetView v = views[tk.set];
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (uint32_t q = tid; q < (uint32_t)kLogEntries; q += 1024) log_table_entry((int)q, sh.logt[q]);
  if (tid == 0) sh.ln2 = log(2.0);
  if (tid < 48) sh.racc[tid] = 0;
  clear_rows(sh.row);

  const uint32_t ga = tk.g0 + wave, gb = tk.g0 + 31u - wave;
#pragma unroll
  for (int k = 0; k < 6; k++) (&sh.colacc[wave][0][0][0])[k * 64 + lane] = 0;

  for (uint32_t rb = tk.rb0; rb < tk.rb1; rb++) {
    if (rb > tk.rb0) {
      // previous row block: flush its row sums, then remove it from the table
      const uint32_t pr = rb - 1;
      if (tid < 48) {
        const uint32_t s = 16u * pr + tid / 3u;
        if (s < v.N)
          atomicAdd(reinterpret_cast<unsigned long long *>(v.acc) + 3ull * s + tid % 3u, sh.racc[tid]);
        sh.racc[tid] = 0;
      }
      touch_rows<false>(v, ConsecutiveRows{16u * pr, v.N}, v.exc_ids, v.exc_off[pr], v.exc_n[pr], sh.row);
    }
    __syncthreads();
    const uint32_t e0 = v.exc_off[rb], en = v.exc_n[rb];
    touch_rows<true>(v, ConsecutiveRows{16u * rb, v.N}, v.exc_ids, e0, en, sh.row);
    const bool lds_exc = en <= kExcLds;
    if (lds_exc) {
      for (uint32_t e = tid; e < en; e += 1024) sh.exc_id[e] = v.exc_ids[e0 + e];
      for (uint32_t e = tid; e < 16u * en; e += 1024) sh.exc_c[e] = v.exc_cnt[16ull * e0 + e];
    }
    __syncthreads();
    const uint16_t *eid = lds_exc ? sh.exc_id : v.exc_ids + e0;
    const uint16_t *ecnt = lds_exc ? sh.exc_c : v.exc_cnt + 16ull * e0;
    // a tile has pairs below the diagonal only when rb >= 4 g
    if (ga < v.G && rb >= 4u * ga)
      rank_tile<false>(v, sh, rb, ga, v.N, delta, eid, ecnt, en, sh.colacc[wave][0]);
    if (gb < v.G && rb >= 4u * gb)
      rank_tile<false>(v, sh, rb, gb, v.N, delta, eid, ecnt, en, sh.colacc[wave][1]);
    __syncthreads();
  }
  if (tid < 48) {
    const uint32_t s = 16u * (tk.rb1 - 1) + tid / 3u;
    if (s < v.N)
      atomicAdd(reinterpret_cast<unsigned long long *>(v.acc) + 3ull * s + tid % 3u, sh.racc[tid]);
  }
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(v.acc);
#pragma unroll
  for (uint32_t gi = 0; gi < 2; gi++) {
    const uint32_t g = gi ? gb : ga, sc = 64u * g + lane;
    if (g < v.G && sc < v.N && tk.rb1 > 4u * g) {
#pragma unroll
      for (int k = 0; k < 3; k++)
        atomicAdd(acc + 3ull * sc + k, (unsigned long long)sh.colacc[wave][gi][k][lane]);
    }
  }
}

hipError_t launch_rank_pairs(hipStream_t st, const SetView *d_views, const PairTask *tasks,
                             uint32_t ntasks, double delta) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_pairs_kernel, dim3(ntasks), dim3(1024), 0, st, d_views, tasks, delta);
  return hipGetLastError();
}

// R = (sum of the pair terms + the j = i term) / N for every sorted
// position of every set; written at the sequence's input index.
__global__ void rank_finalize_kernel(Segs sg, uint32_t N, double delta, double *__restrict__ ranks) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const uint32_t set = sg.set_of_pos(p);
  const uint32_t a = sg.seq[set], n = sg.seq[set + 1] - a;
  const SetView &v = sg.views[set];
  long long *acc = v.acc + 3ull * (p - a);
  long long l0, l1, l2;
  fix_limbs(-log(delta + 1.0), l0, l1, l2);  // the j = i term: F = 1
  const double sum = fix_to_double(acc[0] + l0, acc[1] + l1, acc[2] + l2);
  ranks[a + v.perm[p - a]] = sum / (double)n;
  acc[0] = acc[1] = acc[2] = 0;  // cleared for the next rank launch
}

hipError_t launch_rank_finalize(hipStream_t st, const Segs &sg, uint32_t N, double delta,
                                double *ranks) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_finalize_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sg, N, delta,
                     ranks);
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
  column_excess(v, sc, sh.BM, exc_ids, exc_cnt, e0, en, cnt);
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
