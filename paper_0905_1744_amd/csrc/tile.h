// Tile machinery shared by the rank kernels (pair.hip: all pairs of one
// set; cross.hip: a set against gathered samples).  How a 16-row block
// and a 64-column group meet is described at the top of pair.hip.
#pragma once

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

// Loads through a global-address-space pointer: they count only as vector
// memory operations, so a wait for LDS results does not also wait for them
// (a generic-pointer load counts as both).
__device__ __forceinline__ uint4 gld(const uint4 *p) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(1))) const v4u gv4u;
  const v4u v = *(gv4u *)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}

// 2k masks of the words in x[0..k) (low half first): all 2k LDS reads are
// issued before the first use, so their latencies overlap
template <int K>
__device__ __forceinline__ void lookup_batch(const uint16_t *T16, const uint32_t (&x)[K],
                                             uint32_t (&lo)[K], uint32_t (&hi)[K]) {
#pragma unroll
  for (int k = 0; k < K; k++) {
    lo[k] = T16[x[k] & 0xFFFFu];
    hi[k] = T16[x[k] >> 16];
  }
}

// Level-1 counts of this lane's column (list length L, a multiple of 16,
// the same for the whole wave) against the 16 rows of the LDS table.
// Chunk k of the column (8 words) is p[64 k].  Per 32-word step: the 32
// lookups are issued together, then the next step's four chunks are
// loaded, then the masks are summed; the load after the last step reads
// into the sentinel slack behind the last group.
template <int NP>
__device__ __forceinline__ void column_counts_uniform(const uint16_t *T16, const uint4 *__restrict__ p,
                                                      uint32_t L, uint32_t (&cnt)[16]) {
  uint32_t P[16];
#pragma unroll
  for (int k = 0; k < 16; k++) P[k] = 0;
  const uint32_t n32 = L >> 5;
  uint4 c0 = gld(p), c1 = gld(p + 64), c2 = gld(p + 128), c3 = gld(p + 192);
  for (uint32_t it = 0; it < n32; it++) {
    const uint32_t x[16] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w,
                            c2.x, c2.y, c2.z, c2.w, c3.x, c3.y, c3.z, c3.w};
    uint32_t lo[16], hi[16];
    lookup_batch<16>(T16, x, lo, hi);
    __builtin_amdgcn_sched_barrier(0);
    const uint4 *q = p + (size_t)(it + 1) * 256;
    c0 = gld(q);
    c1 = gld(q + 64);
    c2 = gld(q + 128);
    c3 = gld(q + 192);
    __builtin_amdgcn_sched_barrier(0);
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 16; k++) w[k] = __builtin_amdgcn_perm(hi[k], lo[k], 0x05040100u);
    add16<NP>(P, w);
  }
  if (L & 16u) {
    const uint32_t x[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    uint32_t lo[8], hi[8];
    lookup_batch<8>(T16, x, lo, hi);
    __builtin_amdgcn_sched_barrier(0);
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; k++) w[k] = __builtin_amdgcn_perm(hi[k], lo[k], 0x05040100u);
    add8<NP>(P, w);
  }
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

// Position of word id in the row block's merged count>=2 list (ascending,
// distinct words): the entries before id's bitmap word (BP) plus the set
// bits below id in that word.  Valid only where id's bit is set.
__device__ __forceinline__ uint32_t merged_index(const uint16_t *BP, uint32_t bw, uint32_t id) {
  return (uint32_t)BP[id >> 5] + (uint32_t)__builtin_popcount(bw & ((1u << (id & 31u)) - 1u));
}

// Levels >= 2 for one column: the column's count>=2 words against the row
// block's merged list (bitmap BM and its word offsets BP in LDS; the
// list's counts exc_cnt in global memory from entry e0 on).
__device__ __forceinline__ void column_excess(const SetView &v, uint32_t sc, const uint32_t *BM,
                                              const uint16_t *BP, const uint16_t *__restrict__ exc_cnt,
                                              uint32_t e0, uint32_t (&cnt)[16]) {
  const uint32_t h0 = v.hi_off[sc], h1 = v.hi_off[sc + 1];
  for (uint32_t h = h0; h < h1; h++) {
    const uint32_t id = v.hi_ids[h], bw = BM[id >> 5];
    if (!((bw >> (id & 31u)) & 1u)) continue;
    const uint32_t cj = v.hi_cnt[h];
    const uint16_t *c = exc_cnt + (size_t)(e0 + merged_index(BP, bw, id)) * 16;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const uint32_t cr = c[r];
      cnt[r] += cr >= 2u ? min(cr, cj) - 1u : 0u;
    }
  }
}

// Levels >= 2 for one column of the rank kernel: the column's count>=2
// entries come from the group-interleaved list (q0..q3 are its first four,
// loaded before the level-1 loop); a hit in the row block's bitmap finds
// its entry of the block's merged list by merged_index, and ecnt (LDS copy
// or HBM, 16 counts per entry) gives the rows' counts.
__device__ __forceinline__ void column_excess_grouped(const uint32_t *__restrict__ hp, uint32_t hl,
                                                      const uint32_t (&q0)[4], const uint32_t *BM,
                                                      const uint16_t *BP, const uint16_t *ecnt,
                                                      uint32_t (&cnt)[16]) {
  uint32_t q[4] = {q0[0], q0[1], q0[2], q0[3]};
  for (uint32_t t = 0; t < hl; t += 4) {
    // the next four entries are in flight while these four are looked up
    uint32_t qn[4] = {0u, 0u, 0u, 0u};
    if (t + 4u < hl) {
#pragma unroll
      for (int k = 0; k < 4; k++) qn[k] = hp[(size_t)(t + 4u + k) * 64];
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t id = q[k] & 0xFFFFu, cj = q[k] >> 16, bw = BM[id >> 5];
      if (cj < 2u || !((bw >> (id & 31u)) & 1u)) continue;
      const uint4 *c4 = reinterpret_cast<const uint4 *>(ecnt + (size_t)merged_index(BP, bw, id) * 16);
      const uint4 lo = c4[0], hi = c4[1];
      const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const uint32_t cr = (w[r >> 1] >> (16 * (r & 1))) & 0xFFFFu;
        cnt[r] += cr >= 2u ? min(cr, cj) - 1u : 0u;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = qn[k];
  }
}

// Lane exchanges of the row-sum butterfly, all register to register (no
// LDS): the two halves of a double move as 32-bit words.
__device__ __forceinline__ uint32_t dlo(double x) { return (uint32_t)__double_as_longlong(x); }
__device__ __forceinline__ uint32_t dhi(double x) { return (uint32_t)((unsigned long long)__double_as_longlong(x) >> 32); }
__device__ __forceinline__ double dmk(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One butterfly step across lanes l and l ^ 32 for two values: lanes below
// 32 return a(l) + a(l + 32), lanes from 32 on b(l - 32) + b(l).
// v_permlane32_swap exchanges the upper half of its first operand with the
// lower half of its second.
__device__ __forceinline__ double fold32(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(dlo(a), dlo(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(dhi(a), dhi(b), false, false);
  return dmk(lo[0], hi[0]) + dmk(lo[1], hi[1]);
}

// The same across lanes l and l ^ 16: v_permlane16_swap exchanges the odd
// 16-lane rows of its first operand with the even rows of its second.
__device__ __forceinline__ double fold16(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(dlo(a), dlo(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(dhi(a), dhi(b), false, false);
  return dmk(lo[0], hi[0]) + dmk(lo[1], hi[1]);
}

// x from lane l ^ m, m in {1, 2, 4, 8}, by DPP moves inside 16-lane rows:
// quad permutations for 1 and 2, rotation by 8 for 8, and for 4 two shifts
// by 4 written to alternate groups of four lanes (bank masks).
template <int M>
__device__ __forceinline__ uint32_t xor_dpp(uint32_t x) {
  if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // quad_perm 1 0 3 2
  if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);  // quad_perm 2 3 0 1
  if constexpr (M == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false);  // row_ror:8
  if constexpr (M == 4) {
    const int t = __builtin_amdgcn_update_dpp((int)x, (int)x, 0x104, 0xF, 0x5, false);  // row_shl:4, lanes 0-3, 8-11
    return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)x, 0x114, 0xF, 0xA, false);   // row_shr:4, lanes 4-7, 12-15
  }
}
template <int M>
__device__ __forceinline__ double xor_lane(double x) {
  return dmk(xor_dpp<M>(dlo(x)), xor_dpp<M>(dhi(x)));
}

// Finishes a fixed halving butterfly over the 64 lanes.  On entry lane l
// holds u8[i] = the pair sum (lanes l, l^32) of value i + 8 (l >> 5); on
// exit lanes 4r..4r+3 return the total of value r over all 64 lanes.  At
// every step a lane adds its own value to its partner's, so the result does
// not depend on how the values travel.
__device__ __forceinline__ double halving_reduce8(const double (&u8)[8], uint32_t lane) {
  double u4[4], u2[2];
  const bool b3 = lane & 8u, b2 = lane & 4u;
  // lanes with bit 4 clear keep value i, the others value i + 4
#pragma unroll
  for (int i = 0; i < 4; i++) u4[i] = fold16(u8[i], u8[i + 4]);
#pragma unroll
  for (int i = 0; i < 2; i++) {
    const double send = b3 ? u4[i] : u4[i + 2];
    const double keep = b3 ? u4[i + 2] : u4[i];
    u2[i] = keep + xor_lane<8>(send);
  }
  const double send = b2 ? u2[0] : u2[1];
  const double keep = b2 ? u2[1] : u2[0];
  double u1 = keep + xor_lane<4>(send);
  u1 += xor_lane<2>(u1);
  u1 += xor_lane<1>(u1);
  return u1;
}

// LDS state of one row block: presence table, count>=2 bitmap with the
// merged-list offset of each of its words, row data.
struct RowShared {
  uint32_t T32[kTableWords];
  uint32_t BM[kBitmapWords];
  uint16_t BP[kBitmapWords];  // entries of the merged list before word w (set words only)
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
    if (kSet) {
      atomicOr(&sh.BM[id >> 5], 1u << (id & 31u));
      // the list ascends: the first entry of each bitmap word records its offset
      if (e == 0 || (uint32_t)(exc_ids[e0 + e - 1] >> 5) != (id >> 5)) sh.BP[id >> 5] = (uint16_t)e;
    } else {
      sh.BM[id >> 5] = 0;
    }
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
constexpr uint32_t kSplitMinWords = 64;  // shortest list slice worth a wave of its own

struct RankShared {
  RowShared row;
  LogEntry logt[kLogEntries];
  double ln2;
  unsigned long long racc[16];  // row sums of the current row block (fixed point)
  alignas(16) uint16_t exc_c[kExcLds * 16];  // the row block's merged counts when they fit
  long long colacc[32][64];     // [group of the strip][lane] column sums (fixed point)
  uint16_t xcnt[16][16][64];    // [wave][row][lane] level-1 counts of a list slice
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
// Level-1 counts of words [w0, w0 + len) of this lane's column in group g
// (w0 and len multiples of 16) against the row block in the LDS table.
__device__ __forceinline__ void slice_counts(const SetView &v, const RankShared &sh, uint32_t g,
                                             uint32_t w0, uint32_t len, uint32_t (&cnt)[16]) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint4 *p = reinterpret_cast<const uint4 *>(v.gids + v.grp_off[g]) + lane + (size_t)(w0 >> 3) * 64;
  column_counts(reinterpret_cast<const uint16_t *>(sh.row.T32), p, len, cnt);
}

// One 16 x 64 tile: row block rb (in LDS) against column group g (this
// wave).  Within one set (kCross false) a pair counts only below the
// diagonal of the sorted order and the tile's row sums go to sh.racc (LDS,
// exact); with rows from another set (kCross true: the gathered samples of
// the globalized rank, row_n of them) every pair counts and only the
// columns gather sums.  Column sums go into the lane's entry of col.
// tile_finish takes the level-1 counts of the whole column list (however
// they were summed) and does the rest; rank_tile does both parts.
// Per-column data of a tile, loaded before the counting so that its
// latency overlaps the lookups: the column's count>=2 list (length hl per
// lane, first four entries q0) and the reciprocal of its k-mer count K.
struct TileCol {
  const uint32_t *hp;
  uint32_t hl;
  uint32_t q0[4];
  double invKc;
};

__device__ __forceinline__ TileCol tile_col(const SetView &v, uint32_t g) {
  const uint32_t lane = threadIdx.x & 63u;
  TileCol c;
  c.hl = __builtin_amdgcn_readfirstlane(v.ghi_len[g]);
  const uint32_t sc = 64u * g + lane;
  const bool vc = sc < v.N;
  c.hp = v.ghi + v.ghi_off[g] + lane;
#pragma unroll
  for (int k = 0; k < 4; k++) c.q0[k] = 0u;
  if (c.hl > 0) {
#pragma unroll
    for (int k = 0; k < 4; k++) c.q0[k] = c.hp[(size_t)k * 64];
  }
  c.invKc = vc ? v.invK[sc] : 0.0;
  return c;
}

template <bool kCross>
__device__ __forceinline__ void tile_finish(const SetView &v, RankShared &sh, uint32_t rb, uint32_t g,
                                            uint32_t row_n, double delta, int fix, const uint16_t *ecnt,
                                            const TileCol &tc,
                                            uint32_t (&cnt)[16], long long (&col)[64]) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t sc = 64u * g + lane;
  const bool vc = sc < v.N;
  const double invKc = tc.invKc;
  column_excess_grouped(tc.hp, tc.hl, tc.q0, sh.row.BM, sh.row.BP, ecnt, cnt);
  // F = shared / min(K_r, K_c) (Equation 1), d = -ln(delta + F) (Equation 2);
  // rows r and r + 8 are formed together and immediately folded across
  // lanes l and l ^ 32 (first step of the halving butterfly).  Every lane
  // evaluates all 16 rows without branching (the argument of the logarithm
  // is at least delta > 0 even for pairs outside the triangle or the set)
  // and keeps 0 where the pair does not count.  The reciprocal of the
  // shorter K is the larger of the two rounded reciprocals (rounding is
  // monotonic; padding rows and columns hold 0).
  double u8[8];
  double colsum = 0.0;
#pragma unroll
  for (int r = 0; r < 8; r++) {
    double d[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const uint32_t rr = r + 8 * h, sr = 16u * rb + rr;
      const bool ok = vc && (kCross || sc < sr) && sr < row_n;
      const double inv = fmax(sh.row.rowInv[rr], invKc);
      const double nl = log_tab<true>(fma((double)cnt[rr], inv, delta), sh.logt, sh.ln2);
      d[h] = ok ? nl : 0.0;
    }
    colsum += d[0];
    colsum += d[1];
    if (!kCross) u8[r] = fold32(d[0], d[1]);
  }
  if (!kCross) {
    const double rowtot = halving_reduce8(u8, lane);
    if ((lane & 3u) == 0) atomicAdd(sh.racc + (lane >> 2), (unsigned long long)fix_q(rowtot, fix));
  }
  col[lane] += fix_q(colsum, fix);
}

template <bool kCross>
__device__ __forceinline__ void rank_tile(const SetView &v, RankShared &sh, uint32_t rb, uint32_t g,
                                          uint32_t row_n, double delta, int fix, const uint16_t *ecnt,
                                          long long (&col)[64]) {
  const uint32_t L = __builtin_amdgcn_readfirstlane(v.grp_len[g]);
  const TileCol tc = tile_col(v, g);
  uint32_t cnt[16];
  slice_counts(v, sh, g, 0u, L, cnt);
  tile_finish<kCross>(v, sh, rb, g, row_n, delta, fix, ecnt, tc, cnt, col);
}

}  // namespace kd
