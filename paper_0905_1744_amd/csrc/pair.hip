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
#include "bitcount.h"
#include "kd_internal.h"
#include "klog.h"

namespace kd {

// one 32-word step: 16 masks per uint4 pair... (see bitcount.h)
// masks of the two words packed in x, as one 32-bit word (low half: x's
// low word); built as a two-element vector so the halves merge with v_perm
__device__ __forceinline__ uint32_t look2(const uint16_t *T16, uint32_t x) {
  typedef __attribute__((ext_vector_type(2))) unsigned short us2;
  us2 v;
  v.x = T16[x & 0xFFFFu];
  v.y = T16[x >> 16];
  return __builtin_bit_cast(uint32_t, v);
}

template <int NP>
__device__ __forceinline__ void step32(const uint16_t *T16, uint32_t (&P)[16], const uint4 &a0,
                                       const uint4 &a1, const uint4 &a2, const uint4 &a3) {
  uint32_t w[16];
  w[0] = look2(T16, a0.x);  w[1] = look2(T16, a0.y);  w[2] = look2(T16, a0.z);  w[3] = look2(T16, a0.w);
  w[4] = look2(T16, a1.x);  w[5] = look2(T16, a1.y);  w[6] = look2(T16, a1.z);  w[7] = look2(T16, a1.w);
  w[8] = look2(T16, a2.x);  w[9] = look2(T16, a2.y);  w[10] = look2(T16, a2.z); w[11] = look2(T16, a2.w);
  w[12] = look2(T16, a3.x); w[13] = look2(T16, a3.y); w[14] = look2(T16, a3.z); w[15] = look2(T16, a3.w);
  add16<NP>(P, w);
}

template <int NP>
__device__ __forceinline__ void step16(const uint16_t *T16, uint32_t (&P)[16], const uint4 &a0,
                                       const uint4 &a1) {
  uint32_t w[8];
  w[0] = look2(T16, a0.x); w[1] = look2(T16, a0.y); w[2] = look2(T16, a0.z); w[3] = look2(T16, a0.w);
  w[4] = look2(T16, a1.x); w[5] = look2(T16, a1.y); w[6] = look2(T16, a1.z); w[7] = look2(T16, a1.w);
  add8<NP>(P, w);
}

__device__ __forceinline__ void planes_to_counts(uint32_t (&P)[16], uint32_t (&cnt)[16]) {
  transpose16(P);
  typedef __attribute__((ext_vector_type(2))) unsigned short us2;
  const us2 ones = __builtin_bit_cast(us2, 0x00010001u);
#pragma unroll
  for (int r = 0; r < 16; r++)
    cnt[r] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, P[r]), ones, 0u, false);
}

// Level-1 counts of this lane's column (list length L, a multiple of 16,
// the same for the whole wave) against the 16 rows of the LDS table.
// Chunk k of the column (8 words) is p[64 k].  Loads run up to two 32-word
// steps ahead; the word buffer carries enough sentinel slack after the last
// group for that.
template <int NP>
__device__ __forceinline__ void column_counts_uniform(const uint16_t *T16, const uint4 *__restrict__ p,
                                                      uint32_t L, uint32_t (&cnt)[16]) {
  uint32_t P[16];
#pragma unroll
  for (int k = 0; k < 16; k++) P[k] = 0;
  const uint32_t n32 = L >> 5;
  uint4 a0 = p[0], a1 = p[64], a2 = p[128], a3 = p[192];
  uint32_t it = 0;
  for (; it + 2 <= n32; it += 2) {
    const uint4 *q = p + (size_t)(it + 1) * 256;
    const uint4 b0 = q[0], b1 = q[64], b2 = q[128], b3 = q[192];
    step32<NP>(T16, P, a0, a1, a2, a3);
    q += 256;
    a0 = q[0];
    a1 = q[64];
    a2 = q[128];
    a3 = q[192];
    step32<NP>(T16, P, b0, b1, b2, b3);
  }
  if (it < n32) {
    const uint4 *q = p + (size_t)(it + 1) * 256;
    const uint4 b0 = q[0], b1 = q[64];
    step32<NP>(T16, P, a0, a1, a2, a3);
    a0 = b0;
    a1 = b1;
  }
  if (L & 16u) step16<NP>(T16, P, a0, a1);
  planes_to_counts(P, cnt);
}

// Same for lanes whose columns have different list lengths (L_lane, the
// wave's longest being L_wave); chunks past L_lane read as sentinels.
template <int NP>
__device__ __forceinline__ void column_counts_ragged(const uint16_t *T16, const uint4 *__restrict__ p,
                                                     uint32_t L_lane, uint32_t L_wave,
                                                     uint32_t (&cnt)[16]) {
  uint32_t P[16];
#pragma unroll
  for (int k = 0; k < 16; k++) P[k] = 0;
  const uint4 sent = make_uint4(0xB640B640u, 0xB640B640u, 0xB640B640u, 0xB640B640u);
  const uint32_t nchunk = L_lane >> 3;
  uint32_t k = 0;
  for (; k + 4 <= (L_wave >> 3); k += 4) {
    const uint4 a0 = k < nchunk ? p[(size_t)k * 64] : sent;
    const uint4 a1 = k + 1 < nchunk ? p[(size_t)(k + 1) * 64] : sent;
    const uint4 a2 = k + 2 < nchunk ? p[(size_t)(k + 2) * 64] : sent;
    const uint4 a3 = k + 3 < nchunk ? p[(size_t)(k + 3) * 64] : sent;
    step32<NP>(T16, P, a0, a1, a2, a3);
  }
  if (k < (L_wave >> 3)) {
    const uint4 a0 = k < nchunk ? p[(size_t)k * 64] : sent;
    const uint4 a1 = k + 1 < nchunk ? p[(size_t)(k + 1) * 64] : sent;
    step16<NP>(T16, P, a0, a1);
  }
  planes_to_counts(P, cnt);
}

// plane-count bucket of a list length L (counters see at most L/2 words)
__device__ __forceinline__ int np_bucket(uint32_t L) {
  const int need = planes_for(L >> 1);
  return need <= 8 ? 8 : need <= 10 ? 10 : need <= 12 ? 12 : need <= 14 ? 14 : 16;
}

// Levels >= 2 for one column: the column's count>=2 words against the row
// block's merged list (bitmap BM in LDS; exc_* in global memory).
__device__ __forceinline__ void column_excess(const SetView &v, uint32_t sc, const uint32_t *BM,
                                              const uint16_t *__restrict__ exc_ids,
                                              const uint16_t *__restrict__ exc_cnt, uint32_t e0,
                                              uint32_t en, uint32_t (&cnt)[16]) {
  const uint32_t h0 = v.hi_off[sc], h1 = v.hi_off[sc + 1];
  for (uint32_t h = h0; h < h1; h++) {
    const uint32_t id = v.hi_ids[h];
    if (!((BM[id >> 5] >> (id & 31u)) & 1u)) continue;
    const uint32_t cj = v.hi_cnt[h];
    uint32_t lo = e0, hi = e0 + en;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (exc_ids[mid] < id) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= e0 + en || exc_ids[lo] != id) continue;  // not expected: bitmap built from the list
    const uint16_t *c = exc_cnt + (size_t)lo * 16;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const uint32_t cr = c[r];
      cnt[r] += cr >= 2u ? min(cr, cj) - 1u : 0u;
    }
  }
}

// Levels >= 2 for one column of the rank kernel: the column's count>=2
// entries come from the group-interleaved list (q0..q3 are its first four,
// loaded before the level-1 loop); hits in the row block's bitmap are
// looked up in the block's merged list (eid/ecnt: LDS copy or HBM).
__device__ __forceinline__ void column_excess_grouped(const uint32_t *__restrict__ hp, uint32_t hl,
                                                      const uint32_t (&q0)[4], const uint32_t *BM,
                                                      const uint16_t *eid, const uint16_t *ecnt,
                                                      uint32_t en, uint32_t (&cnt)[16]) {
  for (uint32_t t = 0; t < hl; t += 4) {
    uint32_t q[4];
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = t == 0 ? q0[k] : hp[(size_t)(t + k) * 64];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t id = q[k] & 0xFFFFu, cj = q[k] >> 16;
      if (cj < 2u || !((BM[id >> 5] >> (id & 31u)) & 1u)) continue;
      uint32_t lo = 0, hi = en;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (eid[mid] < id) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= en || eid[lo] != id) continue;
      const uint16_t *c = ecnt + (size_t)lo * 16;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const uint32_t cr = c[r];
        cnt[r] += cr >= 2u ? min(cr, cj) - 1u : 0u;
      }
    }
  }
}

// Finishes a fixed halving butterfly over the 64 lanes.  On entry lane l
// holds u8[i] = the pair sum (lanes l, l^32) of value i + 8 (l >> 5); on
// exit lanes 4r..4r+3 return the total of value r over all 64 lanes.
__device__ __forceinline__ double halving_reduce8(const double (&u8)[8], uint32_t lane) {
  double u4[4], u2[2];
  const bool b4 = lane & 16u, b3 = lane & 8u, b2 = lane & 4u;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const double send = b4 ? u8[i] : u8[i + 4];
    const double keep = b4 ? u8[i + 4] : u8[i];
    u4[i] = keep + __shfl_xor(send, 16, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const double send = b3 ? u4[i] : u4[i + 2];
    const double keep = b3 ? u4[i + 2] : u4[i];
    u2[i] = keep + __shfl_xor(send, 8, 64);
  }
  const double send = b2 ? u2[0] : u2[1];
  const double keep = b2 ? u2[1] : u2[0];
  double u1 = keep + __shfl_xor(send, 4, 64);
  u1 += __shfl_xor(u1, 2, 64);
  u1 += __shfl_xor(u1, 1, 64);
  return u1;
}

// LDS state of one row block: presence table, count>=2 bitmap, row data.
struct RowShared {
  uint32_t T32[kTableWords];
  uint32_t BM[kBitmapWords];
  uint32_t rowK[16];
  double rowInv[16];
};

// Inserts (set = true) or removes the rows rowpos(r) (sorted positions,
// 0xFFFFFFFF = none) and their count>=2 words.  Needs 1024 threads: wave r
// walks row r.  Removal zeroes whole entries, which is exact because the
// table holds only the rows being removed.
template <bool kSet, class RowPos>
__device__ __forceinline__ void touch_rows(const SetView &v, RowPos rowpos,
                                           const uint16_t *__restrict__ exc_ids, uint32_t e0,
                                           uint32_t en, RowShared &sh) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t r = wave, sr = rowpos(r);
  uint16_t *T16 = reinterpret_cast<uint16_t *>(sh.T32);
  if (sr != 0xFFFFFFFFu) {
    const uint32_t g = sr >> 6, ln = sr & 63u, Dr = v.D[sr];
    const uint16_t *base = v.gids + v.grp_off[g];
    for (uint32_t t = lane; t < Dr; t += 64) {
      const uint32_t id = base[((size_t)(t >> 3) * 64 + ln) * 8 + (t & 7u)];
      if (kSet) atomicOr(&sh.T32[id >> 1], (1u << r) << ((id & 1u) << 4));
      else T16[id] = 0;
    }
  }
  if (kSet && lane == 0) {
    sh.rowK[r] = sr != 0xFFFFFFFFu ? v.K[sr] : 0u;
    sh.rowInv[r] = sr != 0xFFFFFFFFu ? v.invK[sr] : 0.0;
  }
  for (uint32_t e = tid; e < en; e += 1024) {
    const uint32_t id = exc_ids[e0 + e];
    if (kSet) atomicOr(&sh.BM[id >> 5], 1u << (id & 31u));
    else sh.BM[id >> 5] = 0;
  }
}

__device__ __forceinline__ void clear_rows(RowShared &sh) {
  for (uint32_t x = threadIdx.x; x < (uint32_t)kTableWords; x += blockDim.x) sh.T32[x] = 0;
  for (uint32_t x = threadIdx.x; x < (uint32_t)kBitmapWords; x += blockDim.x) sh.BM[x] = 0;
}

struct ConsecutiveRows {
  uint32_t s0, N;
  __device__ uint32_t operator()(uint32_t r) const { return s0 + r < N ? s0 + r : 0xFFFFFFFFu; }
};

struct ListedRows {
  const uint32_t *pos;
  __device__ uint32_t operator()(uint32_t r) const { return pos[r]; }
};

constexpr uint32_t kExcLds = 256;  // merged count>=2 words of a row block kept in LDS

struct RankShared {
  RowShared row;
  LogEntry logt[kLogEntries];
  double ln2;
  unsigned long long racc[48];  // 16 rows x 3 limbs of the current row block
  uint16_t exc_id[kExcLds];
  uint16_t exc_c[kExcLds * 16];
  long long colacc[16][2][3][64];  // [wave][group of the wave][limb][lane]
};

// Level-1 counts for this lane's column, dispatching on the plane bucket.
__device__ __forceinline__ void column_counts(const uint16_t *T16, const uint4 *p, uint32_t L,
                                              uint32_t (&cnt)[16]) {
  switch (np_bucket(L)) {
    case 8: column_counts_uniform<8>(T16, p, L, cnt); break;
    case 10: column_counts_uniform<10>(T16, p, L, cnt); break;
    case 12: column_counts_uniform<12>(T16, p, L, cnt); break;
    case 14: column_counts_uniform<14>(T16, p, L, cnt); break;
    default: column_counts_uniform<16>(T16, p, L, cnt); break;
  }
}

// One 16 x 64 tile: row block rb (in LDS) against column group g (this
// wave).  Within one set (kCross false) a pair counts only below the
// diagonal of the sorted order and the tile's row sums go to sh.racc (LDS,
// exact); with rows from another set (kCross true: the gathered samples of
// the globalized rank, row_n of them) every pair counts and only the
// columns gather sums.  Column sums go into the lane's limbs.
template <bool kCross>
__device__ __forceinline__ void rank_tile(const SetView &v, RankShared &sh, uint32_t rb, uint32_t g,
                                          uint32_t row_n, double delta, const uint16_t *eid,
                                          const uint16_t *ecnt, uint32_t en, long long (&col)[3][64]) {
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
  const uint32_t Kc = vc ? v.K[sc] : 1u;
  const double invKc = vc ? v.invK[sc] : 0.0;
  uint32_t cnt[16];
  column_counts(reinterpret_cast<const uint16_t *>(sh.row.T32), p, L, cnt);
  column_excess_grouped(hp, hl, q0, sh.row.BM, eid, ecnt, en, cnt);
  // F = shared / min(K_r, K_c) (Equation 1), d = -ln(delta + F) (Equation 2);
  // rows r and r + 8 are formed together and immediately folded across
  // lanes l and l ^ 32 (first step of the halving butterfly)
  double u8[8];
  double colsum = 0.0;
  const bool b5 = lane & 32u;
#pragma unroll
  for (int r = 0; r < 8; r++) {
    double d[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const uint32_t rr = r + 8 * h, sr = 16u * rb + rr;
      d[h] = 0.0;
      if (vc && (kCross || sc < sr) && sr < row_n) {
        const double inv = sh.row.rowK[rr] < Kc ? sh.row.rowInv[rr] : invKc;
        d[h] = -log_tab(fma((double)cnt[rr], inv, delta), sh.logt, sh.ln2);
      }
    }
    colsum += d[0];
    colsum += d[1];
    if (!kCross) {
      const double send = b5 ? d[0] : d[1];
      const double keep = b5 ? d[1] : d[0];
      u8[r] = keep + __shfl_xor(send, 32, 64);
    }
  }
  if (!kCross) {
    const double rowtot = halving_reduce8(u8, lane);
    if ((lane & 3u) == 0) {
      long long l0, l1, l2;
      fix_limbs(rowtot, l0, l1, l2);
      unsigned long long *ra = sh.racc + 3u * (lane >> 2);
      atomicAdd(ra, (unsigned long long)l0);
      atomicAdd(ra + 1, (unsigned long long)l1);
      atomicAdd(ra + 2, (unsigned long long)l2);
    }
  }
  long long l0, l1, l2;
  fix_limbs(colsum, l0, l1, l2);
  col[0][lane] += l0;
  col[1][lane] += l1;
  col[2][lane] += l2;
}

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

  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t ga = __builtin_amdgcn_readfirstlane(gperm[tk.gx0 + wave]);
  const uint32_t gb = gpt == 32u ? __builtin_amdgcn_readfirstlane(gperm[tk.gx0 + 31u - wave]) : kNone;
#pragma unroll
  for (int k = 0; k < 6; k++) (&sh.colacc[wave][0][0][0])[k * 64 + lane] = 0;

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
      for (uint32_t e = tid; e < en; e += 1024) sh.exc_id[e] = rv.exc_ids[e0 + e];
      for (uint32_t e = tid; e < 16u * en; e += 1024) sh.exc_c[e] = rv.exc_cnt[16ull * e0 + e];
    }
    __syncthreads();
    const uint16_t *eid = lds_exc ? sh.exc_id : rv.exc_ids + e0;
    const uint16_t *ecnt = lds_exc ? sh.exc_c : rv.exc_cnt + 16ull * e0;
    if (ga != kNone) {
      uint32_t gl;
      const uint32_t q = cross_set(cols, ga, gl);
      rank_tile<true>(cols.views[q], sh, rb, gl, rv.N, delta, eid, ecnt, en, sh.colacc[wave][0]);
    }
    if (gb != kNone) {
      uint32_t gl;
      const uint32_t q = cross_set(cols, gb, gl);
      rank_tile<true>(cols.views[q], sh, rb, gl, rv.N, delta, eid, ecnt, en, sh.colacc[wave][1]);
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
    if (sc < v.N) {
      unsigned long long *acc = reinterpret_cast<unsigned long long *>(v.acc);
#pragma unroll
      for (int k = 0; k < 3; k++)
        atomicAdd(acc + 3ull * sc + k, (unsigned long long)sh.colacc[wave][h][k][lane]);
    }
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
__global__ void cross_finalize_kernel(Segs sg, uint32_t N, uint32_t S, double *__restrict__ ranks) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const uint32_t set = sg.set_of_pos(p);
  const uint32_t a = sg.seq[set];
  const SetView &v = sg.views[set];
  long long *acc = v.acc + 3ull * (p - a);
  ranks[a + v.perm[p - a]] = fix_to_double(acc[0], acc[1], acc[2]) / (double)S;
  acc[0] = acc[1] = acc[2] = 0;
}

hipError_t launch_cross_finalize(hipStream_t st, const Segs &sg, uint32_t N, uint32_t S,
                                 double *ranks) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(cross_finalize_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sg, N, S,
                     ranks);
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
