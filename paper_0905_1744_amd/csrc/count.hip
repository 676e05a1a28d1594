// k-mer counting (paper Section 3, "k-mer Rank": the count vector c^X of a
// sequence over the epsilon = 6^6 words).
//
// Output per input sequence i, at capacity offset offsets[i] - 5i (the sum
// of K = n - 5 over the sequences before it, so no scan is needed): its
// distinct words in increasing order with their counts, plus D (distinct
// words), K and the number of words seen at least twice.
//
// Four paths by the size of a sequence (n residues, K = n - 5 words):
//  * n <= 1024: one wave, the words in registers, sorted by a bitonic
//    network (count_wave); in a set of at least 64 x the bitmap pass's
//    resident waves (196,608 sequences on 256 compute units) only n <= 256,
//    and 256 < n <= 1024 one wave with a presence bitmap in the wave's LDS
//    area (count_bitmap);
//  * n > 1024 and K <= 4096: one 256-thread workgroup, a presence bitmap in
//    LDS (count_one);
//  * longer sequences (rare): a persistent kernel that histograms into a
//    dense 46656-bin LDS table (two 16-bit bins per word; a sequence has at
//    most 65535 words, so a bin never carries).
#include <algorithm>

#include "radix.h"

namespace kd {

__device__ inline unsigned long long pack_err(uint32_t seq, uint32_t code, uint64_t pos) {
  uint64_t p = pos < (1ull << 28) ? pos : (1ull << 28) - 1;
  return ((unsigned long long)seq << 32) | ((unsigned long long)code << 28) | p;
}

// Validate the offsets of sequence i; returns an error code or kErrNone.
__device__ inline uint32_t check_offsets(const uint64_t *off, uint32_t i, uint32_t N, uint64_t nres,
                                         uint64_t &o0, uint64_t &o1) {
  o0 = off[i];
  o1 = off[i + 1];
  if (o1 < o0 || o1 > nres || (i + 1 == N && o1 != nres) || (i == 0 && o0 != 0)) return kErrInval;
  if (o1 - o0 < (uint64_t)kK) return kErrShort;
  if (o1 - o0 - (kK - 1) > 65535ull) return kErrLong;
  return kErrNone;
}

// Counts one sequence of K <= CAP words with one workgroup of NT threads
// (the second pass, for sequences too long for one wave's registers).
//
// Every word sets its bit in a 46656-bit LDS bitmap; a word whose bit was
// already set is appended to a list of repeats.  Thread t then owns bitmap
// words [6 t, 6 t + 6): a block prefix sum of their popcounts gives each
// thread the rank of its first set bit, so walking its bits in order puts
// the distinct words, already sorted, into an LDS list.  A repeat's rank is
// the prefix of its bitmap chunk plus the popcounts before it; its count
// slot is incremented.  Words and counts then leave with coalesced stores.
constexpr uint32_t kCountThreads = 256;
constexpr uint32_t kBmChunk = (kBitmapWords + kCountThreads - 1) / kCountThreads;  // 6

template <int CAP>
struct CountShared {
  uint32_t bm[kBitmapWords];
  uint32_t cnt[CAP / 2];   // two 16-bit counts per word (a count never exceeds K <= 65535)
  uint16_t rep[CAP];       // repeated occurrences
  uint16_t dw[CAP];        // distinct words in increasing order
  uint32_t cpre[kCountThreads];  // rank of the first set bit of each thread's chunk
  uint32_t wsum[kCountThreads / 64];
  uint32_t wred[kCountThreads / 64];
  uint32_t nrep;
  uint8_t codes[CAP + 8];
  uint8_t lut[256];
};

template <int CAP>
__device__ __forceinline__ void count_one(const uint8_t *__restrict__ res, uint64_t nres,
                                          uint32_t i, uint64_t o0,
                                          uint32_t n, uint64_t cap, CountShared<CAP> &sh,
                                          uint16_t *__restrict__ cap_ids,
                                          uint16_t *__restrict__ cap_cnt,
                                          uint32_t *__restrict__ hi_cap, uint32_t *__restrict__ Dout,
                                          uint32_t *__restrict__ Kout,
                                          uint32_t *__restrict__ nhiout, unsigned long long *err) {
  constexpr uint32_t NT = kCountThreads;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t K = n - (kK - 1);
  // residues in aligned 16-byte chunks; a chunk reaching outside the
  // residue buffer is read bytewise
  const uintptr_t sq = (uintptr_t)(res + o0);
  const uintptr_t a0 = sq & ~(uintptr_t)15;
  const uintptr_t lo = (uintptr_t)res, hi = (uintptr_t)res + nres;
  const uint32_t nch = (uint32_t)((sq + n - a0 + 15) >> 4);
  uint32_t bad = 0xFFFFFFFFu;
  for (uint32_t c = tid; c < nch; c += NT) {
    const uintptr_t ca = a0 + 16u * c;
    uint32_t w[4];
    if (ca >= lo && ca + 16 <= hi) {
      const uint4 v = *reinterpret_cast<const uint4 *>(ca);
      w[0] = v.x;
      w[1] = v.y;
      w[2] = v.z;
      w[3] = v.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; q++) {
        w[q] = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const uintptr_t b = ca + 4 * q + k;
          if (b >= lo && b < hi) w[q] |= (uint32_t)(*reinterpret_cast<const uint8_t *>(b)) << (8 * k);
        }
      }
    }
    const int64_t t0 = (int64_t)(ca - sq);  // sequence position of the chunk's first byte
#pragma unroll
    for (int k = 0; k < 16; k++) {
      const int64_t t = t0 + k;
      if (t >= 0 && t < (int64_t)n) {
        const uint8_t cd = sh.lut[(w[k >> 2] >> (8 * (k & 3))) & 0xFFu];
        sh.codes[t] = cd;
        if (cd == 255 && (uint32_t)t < bad) bad = (uint32_t)t;
      }
    }
  }
  for (uint32_t x = tid; x < (uint32_t)kBitmapWords; x += NT) sh.bm[x] = 0;
  for (uint32_t x = tid; x < (K + 1) / 2; x += NT) sh.cnt[x] = 0;
  if (tid == 0) sh.nrep = 0;
#pragma unroll
  for (int o = 32; o; o >>= 1) bad = min(bad, (uint32_t)__shfl_xor((int)bad, o, 64));
  if (lane == 0) sh.wred[wave] = bad;
  __syncthreads();
#pragma unroll
  for (uint32_t w = 0; w < NT / 64; w++) bad = min(bad, sh.wred[w]);
  if (bad != 0xFFFFFFFFu) {
    if (tid == 0) atomicMin(err, pack_err(i, kErrBadResidue, bad));
    return;  // uniform over the workgroup
  }
  for (uint32_t t = tid; t < K; t += NT) {
    const uint8_t *c = sh.codes + t;
    const uint32_t w = c[0] * 7776u + c[1] * 1296u + c[2] * 216u + c[3] * 36u + c[4] * 6u + c[5];
    const uint32_t bit = 1u << (w & 31u);
    if (atomicOr(&sh.bm[w >> 5], bit) & bit) sh.rep[atomicAdd(&sh.nrep, 1u)] = (uint16_t)w;
  }
  __syncthreads();
  const uint32_t x0 = min(tid * kBmChunk, (uint32_t)kBitmapWords);
  const uint32_t x1 = min(x0 + kBmChunk, (uint32_t)kBitmapWords);
  uint32_t local = 0;
  for (uint32_t x = x0; x < x1; x++) local += __popc(sh.bm[x]);
  uint32_t D;
  uint32_t rank = block_exclusive_scan<NT>(local, sh.wsum, D);
  sh.cpre[tid] = rank;
  for (uint32_t x = x0; x < x1; x++) {
    uint32_t m = sh.bm[x];
    while (m) {
      const uint32_t b = __ffs(m) - 1u;
      m &= m - 1u;
      sh.dw[rank++] = (uint16_t)(32u * x + b);
    }
  }
  __syncthreads();
  const uint32_t nrep = sh.nrep;
  for (uint32_t q = tid; q < nrep; q += NT) {
    const uint32_t w = sh.rep[q], x = w >> 5, c = x / kBmChunk;
    uint32_t r = sh.cpre[c];
    for (uint32_t y = c * kBmChunk; y < x; y++) r += __popc(sh.bm[y]);
    r += __popc(sh.bm[x] & ((1u << (w & 31u)) - 1u));
    atomicAdd(&sh.cnt[r >> 1], 1u << ((r & 1u) << 4));
  }
  __syncthreads();
  const uint64_t co = o0 - 5ull * i;
  const bool ok = (o0 >= 5ull * i) && (co + K <= cap);
  // words and counts; the entries with count >= 2 are also compacted, in
  // word order, into hi_cap (word | count << 16) at the same offset
  uint32_t nh = 0;
  for (uint32_t r0 = 0; r0 < D; r0 += NT) {
    const uint32_t r = r0 + tid;
    uint32_t c = 0;
    if (r < D) {
      c = 1u + ((sh.cnt[r >> 1] >> ((r & 1u) << 4)) & 0xFFFFu);
      if (ok) {
        cap_ids[co + r] = sh.dw[r];
        cap_cnt[co + r] = (uint16_t)c;
      }
    }
    const unsigned long long m = __ballot(c >= 2);
    if (lane == 0) sh.wred[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = nh, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < NT / 64; w++) {
      before += w < wave ? sh.wred[w] : 0u;
      tot += sh.wred[w];
    }
    if (c >= 2 && ok) hi_cap[co + before + (uint32_t)__popcll(m & lanemask_lt())] = sh.dw[r] | (c << 16);
    nh += tot;
    __syncthreads();
  }
  if (tid == 0) {
    Dout[i] = D;
    Kout[i] = K;
    nhiout[i] = nh;
  }
}

// ------------------------------------------------------------------------
// Register-resident counting of one sequence of n <= 64 E residues by one
// wave: lane l forms words E l .. E l + E - 1 from its residues (and the
// following lanes' first five codes), the 64 E words are sorted across the
// wave with a bitonic network (in-register stages for partners inside a
// lane, lane shuffles otherwise), and runs of equal words give the distinct
// words and their counts in order.  LDS holds only the residue table.

constexpr uint32_t kPadWord = 0xFFFFu;  // above every word: sorts last
constexpr uint32_t kWaveMaxLen = 1024;  // longest sequence (in residues) counted by one wave

// Inclusive prefix sum over the wave by DPP moves (no LDS): shifts by 1, 2,
// 4 and 8 inside each 16-lane row, then row 0's total into row 1 and row
// 2's into row 3 (row_bcast:15), then rows 0-1's total into rows 2 and 3
// (row_bcast:31).  Lanes whose source is outside the row add 0.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// Two 16-bit words per register: one packed min or max orders two pairs.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 swap16(u16x2 x) { return __builtin_shufflevector(x, x, 1, 0); }
// The value of lane (lane ^ m).  With m known at compile time (the sort's
// loops are unrolled) the partners inside a quad or a row come by DPP moves
// (quad permutations for 1, 2 and 3, the half-row and row mirrors for 7
// and 15: register to register); the others by a lane shuffle.
__device__ __forceinline__ int lane_xor(int x, int m) {
  switch (m) {
    case 1: return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);   // quad_perm 1 0 3 2
    case 2: return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);   // quad_perm 2 3 0 1
    case 3: return __builtin_amdgcn_mov_dpp(x, 0x1B, 0xF, 0xF, false);   // quad_perm 3 2 1 0
    case 7: return __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    case 15: return __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false); // row_mirror
    default: return __shfl_xor(x, m, 64);
  }
}
__device__ __forceinline__ u16x2 shfl_xor16(u16x2 x, int m) {
  return __builtin_bit_cast(u16x2, lane_xor(__builtin_bit_cast(int, x), m));
}

// The bitonic network of count_wave on 64 E words (E >= 2) held two per
// register: element s of a lane sits in register s mod E/2, in the low half
// when s < E/2.  In-lane partners that differ in the E/2 bit of s meet
// across halves (one register's halves swapped, then the low half of the
// minimum and the high half of the maximum kept); all others meet half to
// half.  A partner in another lane arrives by one shuffle per register,
// halves swapped when the partner is the mirror element E - 1 - s.
template <int E>
__device__ __forceinline__ void bitonic_packed(uint32_t (&v)[E], uint32_t lane) {
  constexpr int H = E / 2;
  u16x2 P[H];
#pragma unroll
  for (int h = 0; h < H; h++) P[h] = u16x2{(unsigned short)v[h], (unsigned short)v[h + H]};
#pragma unroll
  for (uint32_t k = 2; k <= 64u * E; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const uint32_t m = (j == (k >> 1)) ? (k - 1) : j;  // partner = x ^ m
      if (m < (uint32_t)E) {
        if ((m & (uint32_t)H) == 0) {
#pragma unroll
          for (int h = 0; h < H; h++) {
            const int g = h ^ (int)m;
            if (h < g) {
              const u16x2 a = P[h], b = P[g];
              P[h] = __builtin_elementwise_min(a, b);
              P[g] = __builtin_elementwise_max(a, b);
            }
          }
        } else {
          const int mp = (int)m ^ H;
#pragma unroll
          for (int h = 0; h < H; h++) {
            const int g = h ^ mp;
            if (h <= g) {
              const u16x2 a = P[h], sw = swap16(P[g]);
              const u16x2 mn = __builtin_elementwise_min(a, sw), mx = __builtin_elementwise_max(a, sw);
              P[h] = __builtin_shufflevector(mn, mx, 0, 3);
              if (h < g) P[g] = __builtin_shufflevector(mn, mx, 1, 2);
            }
          }
        }
      } else {
        const int lm = (int)(m / E);
        const bool lower = (lane & (j / E)) == 0;
        u16x2 o[H];
#pragma unroll
        for (int h = 0; h < H; h++)
          o[h] = (m == j) ? shfl_xor16(P[h], lm) : swap16(shfl_xor16(P[H - 1 - h], lm));
#pragma unroll
        for (int h = 0; h < H; h++)
          P[h] = lower ? __builtin_elementwise_min(P[h], o[h]) : __builtin_elementwise_max(P[h], o[h]);
      }
    }
  }
#pragma unroll
  for (int h = 0; h < H; h++) {
    v[h] = P[h].x;
    v[h + H] = P[h].y;
  }
}

// Words E lane .. E lane + E - 1 of a sequence of n residues (kPadWord at
// and past K = n - 5).  Each lane maps its own E residues through the
// 256-entry group table lut (7: not one of the 20 amino acids) into 3-bit
// codes, the first in the low bits; the five codes after them come from the
// following lanes by DPP shifts.  The caller takes n <= 64 E, so the zeros
// that lane 63 receives enter only padding words.  Word s + 1 follows
// from word s by dropping its leading base-6 digit and appending the next
// code.  A residue at or past n reads residue n - 1 instead, so its code is
// valid whenever the sequence is; the words it enters are padding.  Returns
// false, after recording the first position that is not an amino acid, when
// there is one (uniform over the wave).
template <int E>
__device__ __forceinline__ bool wave_words(const uint8_t *__restrict__ res, const uint8_t *lut,
                                           uint32_t i, uint64_t o0, uint32_t n, uint32_t lane,
                                           uint32_t (&v)[E], unsigned long long *err) {
  static_assert(E >= 1 && 3 * (E + 5) <= 64, "codes of a lane and the five after them fit 64 bits");
  const uint32_t K = n - (kK - 1);
  const uint32_t t0 = lane * E;
  const uint8_t *p = res + o0;
  uint64_t win = 0;
#pragma unroll
  for (int u = 0; u < E; u++) win |= (uint64_t)lut[p[min(t0 + (uint32_t)u, n - 1)]] << (3 * u);
  // a code is 7 exactly when its three bits are set
  constexpr uint64_t kLow = 0x9249249249249249ull & ((1ull << (3 * E)) - 1);  // bit 0 of each code
  const uint64_t sev = win & (win >> 1) & (win >> 2) & kLow;
  if (__ballot(sev != 0)) {  // rare: the first bad position
    uint32_t bad = 0xFFFFFFFFu;
    if (sev) bad = t0 + (uint32_t)__builtin_ctzll(sev) / 3u;
    bad = bad < n ? bad : 0xFFFFFFFFu;  // (a clamped read repeats residue n - 1)
#pragma unroll
    for (int o = 32; o; o >>= 1) bad = min(bad, (uint32_t)__shfl_xor((int)bad, o, 64));
    if (lane == 0) atomicMin(err, pack_err(i, kErrBadResidue, bad));
    return false;
  }
  // the five codes after this lane's E: lane + 1's first min(E, 5), then
  // lane + 2's, ...
  uint32_t nxt = (uint32_t)win;
#pragma unroll
  for (int got = 0; got < 5; got += E) {
    nxt = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)nxt, 0x130, 0xF, 0xF, false);  // wave_shl:1
    const int take = 5 - got < E ? 5 - got : E;
    win |= (uint64_t)(nxt & ((1u << (3 * take)) - 1u)) << (3 * (E + got));
  }
  uint32_t cd[E + 5];
#pragma unroll
  for (int j = 0; j < E + 5; j++) cd[j] = (uint32_t)(win >> (3 * j)) & 7u;
  uint32_t w = cd[0] * 7776u + cd[1] * 1296u + cd[2] * 216u + cd[3] * 36u + cd[4] * 6u + cd[5];
#pragma unroll
  for (int s = 0; s < E; s++) {
    if (s) w = (w - cd[s - 1] * 7776u) * 6u + cd[s + 5];
    v[s] = t0 + s < K ? w : kPadWord;
  }
  return true;
}

template <int E>
__device__ __forceinline__ void count_wave(const uint8_t *__restrict__ res, const uint8_t *lut,
                                           uint32_t i, uint64_t o0,
                                           uint32_t n, uint64_t cap, uint16_t *__restrict__ cap_ids,
                                           uint16_t *__restrict__ cap_cnt,
                                           uint32_t *__restrict__ hi_cap,
                                           uint32_t *__restrict__ Dout, uint32_t *__restrict__ Kout,
                                           uint32_t *__restrict__ nhiout, unsigned long long *err) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t K = n - (kK - 1);
  const uint32_t t0 = lane * E;
  uint32_t v[E];
  if (!wave_words<E>(res, lut, i, o0, n, lane, v, err)) return;
  // Bitonic sort of the 64 E words, element index x = E lane + s, in the
  // form where every comparator puts the minimum at the lower index: each
  // merge of size k starts by comparing x with its mirror x ^ (k - 1), then
  // halves with x ^ j.
  if constexpr (E >= 2) {
    bitonic_packed<E>(v, lane);
  } else {
    // one word per lane: every partner is in another lane
#pragma unroll
    for (uint32_t k = 2; k <= 64u; k <<= 1) {
#pragma unroll
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        const uint32_t m = (j == (k >> 1)) ? (k - 1) : j;
        const bool lower = (lane & j) == 0;
        const uint32_t o = (uint32_t)lane_xor((int)v[0], (int)m);
        v[0] = lower ? min(v[0], o) : max(v[0], o);
      }
    }
  }
  // runs: a start is an element unlike its predecessor (words sit in
  // [0, K), padding after); a run ends at the next start or at K
  const uint32_t prev_last = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[E - 1], 0x138, 0xF, 0xF, false);  // wave_shr:1
  uint32_t st = 0;  // bit s: element s starts a run
#pragma unroll
  for (int s = 0; s < E; s++) {
    const uint32_t x = t0 + s;
    const uint32_t pv = s ? v[s - 1] : prev_last;
    if (x < K && (x == 0 || v[s] != pv)) st |= 1u << s;
  }
  // first start index in lanes above this one: the lowest such lane's own
  // first start, or K when none
  const uint32_t mine = st ? t0 + (uint32_t)(__ffs(st) - 1) : K;
  const unsigned long long higher = __ballot(st != 0) & ~((2ull << lane) - 1ull);  // lane 63: 0
  const int la = higher ? (int)__builtin_ctzll(higher) : (int)lane;
  const uint32_t from = (uint32_t)__shfl((int)mine, la, 64);
  const uint32_t above = higher ? from : K;
  // positions of the starts and of the count >= 2 starts
  uint32_t cnt[E];
  uint32_t nxt = above, ns = 0, nh = 0;
#pragma unroll
  for (int s = E - 1; s >= 0; s--) {
    const uint32_t x = t0 + s;
    cnt[s] = nxt - x;
    if ((st >> s) & 1u) {
      nxt = x;
      ns++;
      nh += cnt[s] >= 2u;
    }
  }
  const uint32_t ps = wave_incl_sum(ns), ph = wave_incl_sum(nh);
  const uint32_t D = (uint32_t)__builtin_amdgcn_readlane((int)ps, 63);
  const uint32_t NH = (uint32_t)__builtin_amdgcn_readlane((int)ph, 63);
  uint32_t pos = ps - ns, hpos = ph - nh;
  const uint64_t co = o0 - 5ull * i;
  const bool ok = (o0 >= 5ull * i) && (co + K <= cap);
#pragma unroll
  for (int s = 0; s < E; s++) {
    if ((st >> s) & 1u) {
      if (ok) {
        cap_ids[co + pos] = (uint16_t)v[s];
        cap_cnt[co + pos] = (uint16_t)cnt[s];
        if (cnt[s] >= 2u) hi_cap[co + hpos] = v[s] | (cnt[s] << 16);
      }
      pos++;
      hpos += cnt[s] >= 2u;
    }
  }
  if (lane == 0) {
    Dout[i] = D;
    Kout[i] = K;
    nhiout[i] = NH;
  }
}

// ------------------------------------------------------------------------
// Counting of one sequence of kSortMaxLen < n <= kWaveMaxLen residues by one
// wave through a presence bitmap in the wave's own LDS area, without a
// sort.  Every word sets its bit (46656 bits, 1458 words).  Lane l then
// owns bitmap words [24 l, 24 l + 24): their popcounts and a wave prefix
// sum give, for each bitmap word, the number of distinct words below it.
// A word's rank among the distinct words is that number plus the set bits
// below it in its own bitmap word; each occurrence writes its word at its
// rank (equal words write the same value) and adds one to the rank's
// count.  Ranks in increasing order are the words in increasing order, so
// the output (words, counts, the count >= 2 entries) is that of the sort.
// The bitmap words an occurrence set and the counts are cleared after use,
// so the area is clean for the wave's next sequence.
constexpr uint32_t kSortMaxLen = 256;   // longest sequence (in residues) of the register sort
constexpr uint32_t kBmLaneWords = 24;   // bitmap words per lane: 64 x 24 >= 1458

struct alignas(16) BmWave {
  uint32_t bm[64 * kBmLaneWords];   // presence bits; the words past 1458 stay zero
  uint16_t pre[64 * kBmLaneWords];  // distinct words below each bitmap word
  uint16_t dw[kWaveMaxLen];         // distinct words in increasing order
  uint32_t cnt[kWaveMaxLen / 2];    // occurrences per rank, two 16-bit counts per entry
};

// Orders one wave's LDS accesses before and after it: a wave's LDS
// operations reach the LDS in issue order, so a compiler barrier is all
// that is needed for its lanes to see each other's writes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int E>
__device__ __forceinline__ void count_bitmap(const uint8_t *__restrict__ res, const uint8_t *lut,
                                             uint32_t i, uint64_t o0,
                                             uint32_t n, uint64_t cap, BmWave &w,
                                             uint16_t *__restrict__ cap_ids,
                                             uint16_t *__restrict__ cap_cnt,
                                             uint32_t *__restrict__ hi_cap,
                                             uint32_t *__restrict__ Dout, uint32_t *__restrict__ Kout,
                                             uint32_t *__restrict__ nhiout, unsigned long long *err) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t K = n - (kK - 1);
  const uint32_t t0 = lane * E;
  uint32_t v[E];
  if (!wave_words<E>(res, lut, i, o0, n, lane, v, err)) return;
#pragma unroll
  for (int s = 0; s < E; s++)
    if (t0 + s < K) atomicOr(&w.bm[v[s] >> 5], 1u << (v[s] & 31u));
  wave_lds_sync();
  uint32_t b[kBmLaneWords];
  const uint4 *src = reinterpret_cast<const uint4 *>(w.bm + kBmLaneWords * lane);
#pragma unroll
  for (uint32_t q = 0; q < kBmLaneWords / 4; q++) {
    const uint4 x = src[q];
    b[4 * q] = x.x;
    b[4 * q + 1] = x.y;
    b[4 * q + 2] = x.z;
    b[4 * q + 3] = x.w;
  }
  uint32_t below[kBmLaneWords], tot = 0;
#pragma unroll
  for (uint32_t q = 0; q < kBmLaneWords; q++) {
    below[q] = tot;
    tot += (uint32_t)__popc(b[q]);
  }
  const uint32_t incl = wave_incl_sum(tot);
  const uint32_t D = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  const uint32_t base = incl - tot;
  uint2 *dst = reinterpret_cast<uint2 *>(w.pre + kBmLaneWords * lane);
#pragma unroll
  for (uint32_t q = 0; q < kBmLaneWords / 4; q++)
    dst[q] = make_uint2((base + below[4 * q]) | ((base + below[4 * q + 1]) << 16),
                        (base + below[4 * q + 2]) | ((base + below[4 * q + 3]) << 16));
  wave_lds_sync();
  // every read before the first write, so the reads go out together
  uint32_t pw[E], bw[E];
#pragma unroll
  for (int s = 0; s < E; s++) {
    const uint32_t x = min(v[s] >> 5, 64u * kBmLaneWords - 1u);  // padding reads a zero word
    pw[s] = w.pre[x];
    bw[s] = w.bm[x];
  }
#pragma unroll
  for (int s = 0; s < E; s++) {
    if (t0 + s < K) {
      const uint32_t r = pw[s] + (uint32_t)__popc(bw[s] & ((1u << (v[s] & 31u)) - 1u));
      w.dw[r] = (uint16_t)v[s];
      atomicAdd(&w.cnt[r >> 1], 1u << ((r & 1u) << 4));
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int s = 0; s < E; s++)
    if (t0 + s < K) w.bm[v[s] >> 5] = 0u;
  const uint64_t co = o0 - 5ull * i;
  const bool ok = (o0 >= 5ull * i) && (co + K <= cap);
  uint32_t nh = 0;
  for (uint32_t r0 = 0; r0 < D; r0 += 64) {
    const uint32_t r = r0 + lane;
    uint32_t c = 0, wd = 0;
    if (r < D) {
      wd = w.dw[r];
      c = (w.cnt[r >> 1] >> ((r & 1u) << 4)) & 0xFFFFu;
      if (ok) {
        cap_ids[co + r] = (uint16_t)wd;
        cap_cnt[co + r] = (uint16_t)c;
      }
      if ((r & 1u) == 0) w.cnt[r >> 1] = 0u;  // after both ranks of the entry were read
    }
    const unsigned long long m = __ballot(c >= 2);
    if (c >= 2 && ok) hi_cap[co + nh + (uint32_t)__popcll(m & lanemask_lt())] = wd | (c << 16);
    nh += (uint32_t)__popcll(m);
  }
  wave_lds_sync();
  if (lane == 0) {
    Dout[i] = D;
    Kout[i] = K;
    nhiout[i] = nh;
  }
}

// Second pass over the sequences of kSortMaxLen < n <= kWaveMaxLen residues,
// one LDS area per wave.  A wave takes chunks of cs <= 64 consecutive
// sequences: its own, then, in a persistent launch, chunks from a counter.
// One ballot finds a chunk's sequences on this path (re-validating their
// offsets: an invalid sequence was reported by the first pass and is
// skipped), and the wave counts them one after the other.  cs grows with N
// (launch_count), so a small set still spreads its sequences over many
// waves and a large one takes few counter increments.
constexpr uint32_t kBmWavesPerGroup = 4;
constexpr uint32_t kBmGroupsPerCu = 3;  // 3 x 4 x 13 KB of LDS per compute unit

__global__ __launch_bounds__(64 * kBmWavesPerGroup) void count_bitmap_kernel(
    const uint8_t *__restrict__ res, const uint64_t *__restrict__ off, uint32_t N, uint64_t nres,
    uint64_t cap, uint16_t *__restrict__ cap_ids, uint16_t *__restrict__ cap_cnt,
    uint32_t *__restrict__ hi_cap, uint32_t *__restrict__ Dout, uint32_t *__restrict__ Kout,
    uint32_t *__restrict__ nhiout, uint32_t cs, bool persistent, uint32_t *__restrict__ next_chunk,
    unsigned long long *err) {
  __shared__ BmWave area[kBmWavesPerGroup];
  __shared__ uint8_t lut[256];
  for (uint32_t c = threadIdx.x; c < 256; c += blockDim.x) lut[c] = dayhoff6(c) == 255 ? 7 : dayhoff6(c);
  __syncthreads();  // the kernel's only workgroup barrier
  const uint32_t lane = threadIdx.x & 63u;
  BmWave &w = area[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
  for (uint32_t x = lane; x < 64u * kBmLaneWords; x += 64) w.bm[x] = 0u;
  for (uint32_t x = lane; x < kWaveMaxLen / 2; x += 64) w.cnt[x] = 0u;
  wave_lds_sync();
  // the first chunk is the wave's own; a persistent launch continues with
  // chunks from the counter, numbered after the launch's waves
  uint32_t ch = blockIdx.x * kBmWavesPerGroup + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    if ((uint64_t)ch * cs >= N) break;  // every wave ends here once the chunks are taken
    const uint32_t il = ch * cs + lane;
    uint64_t a0 = 0, a1 = 0;
    bool take = false;
    if (lane < cs && il < N && check_offsets(off, il, N, nres, a0, a1) == kErrNone) {
      take = a1 - a0 > kSortMaxLen && a1 - a0 <= kWaveMaxLen;
    }
    unsigned long long m = __ballot(take);
    while (m) {
      const uint32_t j = (uint32_t)__builtin_ctzll(m);
      m &= m - 1ull;
      const uint32_t i = ch * cs + j;
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)a0, j);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(a0 >> 32), j);
      const uint32_t n = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(a1 - a0), j);
      const uint64_t o0 = ((uint64_t)hi << 32) | lo;
      if (kSortMaxLen < 256u && n <= 256u)
        count_bitmap<4>(res, lut, i, o0, n, cap, w, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
      else if (n <= 512u)
        count_bitmap<8>(res, lut, i, o0, n, cap, w, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
      else
        count_bitmap<16>(res, lut, i, o0, n, cap, w, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
    }
    if (!persistent) break;
    uint32_t nx = 0;
    if (lane == 0) nx = atomicAdd(next_chunk, 1u);
    ch = gridDim.x * kBmWavesPerGroup + (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)nx, 0, 64));
  }
}

// First pass, one wave per sequence (four per workgroup): validates every
// sequence, counts in registers those of at most kWaveMaxLen residues (ALL)
// or of at most kSortMaxLen, leaving the others up to kWaveMaxLen to the
// bitmap pass, and queues longer ones for the 4096-word kernel or the
// dense-histogram one.
template <bool ALL>
__global__ __launch_bounds__(256) void count_wave_kernel(
    const uint8_t *__restrict__ res, const uint64_t *__restrict__ off, uint64_t *__restrict__ in_off,
    uint32_t N, uint64_t nres,
    uint64_t cap, uint16_t *__restrict__ cap_ids, uint16_t *__restrict__ cap_cnt,
    uint32_t *__restrict__ hi_cap,
    uint32_t *__restrict__ Dout, uint32_t *__restrict__ Kout, uint32_t *__restrict__ nhiout,
    uint32_t *__restrict__ mid_list, uint32_t *__restrict__ nmid, uint32_t *__restrict__ long_list,
    uint32_t *__restrict__ nlong, unsigned long long *err) {
  __shared__ uint8_t lut[256];
  lut[threadIdx.x] = dayhoff6(threadIdx.x) == 255 ? 7 : dayhoff6(threadIdx.x);
  __syncthreads();  // the kernel's only workgroup barrier
  const uint32_t i = blockIdx.x * 4u + (threadIdx.x >> 6), lane = threadIdx.x & 63u;
  if (i >= N) return;
  uint64_t o0, o1;
  const uint32_t code = check_offsets(off, i, N, nres, o0, o1);
  if (code != kErrNone) {
    if (lane == 0) atomicMin(err, pack_err(i, code, 0));
    return;
  }
  if (lane == 0) {
    in_off[i] = o0;
    if (i + 1 == N) in_off[N] = o1;
  }
  const uint32_t n = (uint32_t)(o1 - o0);
  const uint32_t K = n - (kK - 1);
  if (!ALL && n > kSortMaxLen && n <= kWaveMaxLen) return;  // count_bitmap_kernel's
  if (n > kWaveMaxLen) {
    if (lane == 0) {
      if (K <= (uint32_t)kShortMax) mid_list[atomicAdd(nmid, 1u)] = i;
      else long_list[atomicAdd(nlong, 1u)] = i;
    }
    return;
  }
  if (n <= 64u) count_wave<1>(res, lut, i, o0, n, cap, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
  else if (n <= 128u) count_wave<2>(res, lut, i, o0, n, cap, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
  else if (!ALL || n <= 256u) count_wave<4>(res, lut, i, o0, n, cap, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
  else if (n <= 512u) count_wave<8>(res, lut, i, o0, n, cap, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
  else count_wave<16>(res, lut, i, o0, n, cap, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
}

// Sequences of more than 1024 residues and at most 4096 words, queued by
// the first pass.
__global__ __launch_bounds__(kCountThreads) void count_mid_kernel(
    const uint8_t *__restrict__ res, const uint64_t *__restrict__ off, uint64_t nres, uint64_t cap,
    uint16_t *__restrict__ cap_ids, uint16_t *__restrict__ cap_cnt, uint32_t *__restrict__ hi_cap,
    uint32_t *__restrict__ Dout,
    uint32_t *__restrict__ Kout, uint32_t *__restrict__ nhiout,
    const uint32_t *__restrict__ mid_list, const uint32_t *__restrict__ nmid,
    unsigned long long *err) {
  constexpr int CAP = kShortMax;
  __shared__ CountShared<CAP> sh;
  for (uint32_t c = threadIdx.x; c < 256; c += kCountThreads) sh.lut[c] = dayhoff6(c);
  __syncthreads();
  const uint32_t nm = *nmid;
  for (uint32_t q = blockIdx.x; q < nm; q += gridDim.x) {
    const uint32_t i = mid_list[q];
    const uint64_t o0 = off[i], o1 = off[i + 1];
    count_one<CAP>(res, nres, i, o0, (uint32_t)(o1 - o0), cap, sh, cap_ids, cap_cnt, hi_cap, Dout,
                   Kout, nhiout, err);
    __syncthreads();
  }
}

__global__ __launch_bounds__(1024) void count_long_kernel(
    const uint8_t *__restrict__ res, const uint64_t *__restrict__ off, uint32_t N, uint64_t nres,
    uint64_t cap, uint16_t *__restrict__ cap_ids, uint16_t *__restrict__ cap_cnt,
    uint32_t *__restrict__ hi_cap,
    uint32_t *__restrict__ Dout, uint32_t *__restrict__ Kout, uint32_t *__restrict__ nhiout,
    const uint32_t *__restrict__ long_list, const uint32_t *__restrict__ nlong,
    unsigned long long *err) {
  __shared__ uint32_t hist[kWords / 2];
  __shared__ uint8_t lut[256];
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t s_bad;
  const uint32_t tid = threadIdx.x;
  for (uint32_t c = tid; c < 256; c += 1024) lut[c] = dayhoff6(c);
  const uint32_t nl = *nlong;
  for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
    const uint32_t i = long_list[q];
    const uint64_t o0 = off[i], o1 = off[i + 1];
    const uint32_t n = (uint32_t)(o1 - o0);
    const uint32_t K = n - (kK - 1);
    for (uint32_t x = tid; x < kWords / 2; x += 1024) hist[x] = 0;
    if (tid == 0) s_bad = 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t t = tid; t < n; t += 1024)
      if (lut[res[o0 + t]] == 255) atomicMin(&s_bad, t);
    __syncthreads();
    if (s_bad != 0xFFFFFFFFu) {
      if (tid == 0) atomicMin(err, pack_err(i, kErrBadResidue, s_bad));
      __syncthreads();
      continue;
    }
    for (uint32_t t = tid; t < K; t += 1024) {
      const uint8_t *p = res + o0 + t;
      uint32_t v = lut[p[0]] * 7776u + lut[p[1]] * 1296u + lut[p[2]] * 216u + lut[p[3]] * 36u +
                   lut[p[4]] * 6u + lut[p[5]];
      atomicAdd(&hist[v >> 1], 1u << ((v & 1u) << 4));
    }
    __syncthreads();
    // thread tid owns bins [46 tid, 46 tid + 46)
    const uint32_t b0 = tid * 46u, b1 = min(b0 + 46u, (uint32_t)kWords);
    uint32_t cnt = 0, nh = 0;
    for (uint32_t b = b0; b < b1; b++) {
      const uint32_t c = (hist[b >> 1] >> ((b & 1u) << 4)) & 0xFFFFu;
      cnt += (c != 0);
      nh += (c >= 2);
    }
    uint32_t D, NH;
    uint32_t pos = block_exclusive_scan<1024>(cnt, wsum, D);
    uint32_t hpos = block_exclusive_scan<1024>(nh, wsum, NH);
    const uint64_t co = o0 - 5ull * i;
    const bool ok = (o0 >= 5ull * i) && (co + K <= cap);
    for (uint32_t b = b0; b < b1; b++) {
      const uint32_t c = (hist[b >> 1] >> ((b & 1u) << 4)) & 0xFFFFu;
      if (c) {
        if (ok) {
          cap_ids[co + pos] = (uint16_t)b;
          cap_cnt[co + pos] = (uint16_t)c;
          if (c >= 2) hi_cap[co + hpos] = b | (c << 16);
        }
        pos++;
        hpos += c >= 2;
      }
    }
    if (tid == 0) {
      Dout[i] = D;
      Kout[i] = K;
      nhiout[i] = NH;
    }
    __syncthreads();
  }
}

hipError_t launch_count(hipStream_t st, const uint8_t *res, const uint64_t *off, uint64_t *in_off,
                        uint32_t N, uint64_t nres, uint64_t cap, uint16_t *cap_ids, uint16_t *cap_cnt,
                        uint32_t *hi_cap, uint32_t *Dorig, uint32_t *Korig, uint32_t *nhi_orig,
                        uint32_t *mid_list, uint32_t *nmid, uint32_t *long_list, uint32_t *nlong,
                        uint32_t *next_chunk, unsigned long long *err, int cus) {
  if (N == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)(cus > 0 ? cus : 256);
  // The bitmap pass pays for its own launch only on large sets: from 64 x
  // its resident waves on, sequences of 257..1024 residues go to it; below,
  // the first pass sorts every sequence of up to 1024 residues.  Chunks of
  // cs sequences, about four per wave of a full launch and at most 64.
  // Below 64 every chunk gets a wave of its own (no counter); at 64 the
  // launch is persistent and balances the chunks through the counter.
  const uint32_t bm_waves = kBmGroupsPerCu * grid * kBmWavesPerGroup;
  const bool bitmap = (uint64_t)N >= 64ull * bm_waves;
  if (bitmap)
    hipLaunchKernelGGL(count_wave_kernel<false>, dim3((N + 3) / 4), dim3(256), 0, st, res, off, in_off, N,
                       nres, cap, cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, mid_list, nmid,
                       long_list, nlong, err);
  else
    hipLaunchKernelGGL(count_wave_kernel<true>, dim3((N + 3) / 4), dim3(256), 0, st, res, off, in_off, N,
                       nres, cap, cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, mid_list, nmid,
                       long_list, nlong, err);
  KD_HIP(hipGetLastError());
  if (bitmap) {
    const uint32_t cs = std::max(1u, std::min(64u, N / (4u * bm_waves)));
    const bool persistent = cs == 64u;
    const uint32_t chunks = (N + cs - 1) / cs;
    const uint32_t all_groups = (chunks + kBmWavesPerGroup - 1) / kBmWavesPerGroup;
    const uint32_t bm_grid = persistent ? std::min(kBmGroupsPerCu * grid, all_groups) : all_groups;
    hipLaunchKernelGGL(count_bitmap_kernel, dim3(bm_grid), dim3(64 * kBmWavesPerGroup), 0, st, res, off, N,
                       nres, cap, cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, cs, persistent,
                       next_chunk, err);
    KD_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(count_mid_kernel, dim3(2 * grid), dim3(kCountThreads), 0, st, res, off, nres,
                     cap, cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, mid_list, nmid, err);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(count_long_kernel, dim3(grid), dim3(1024), 0, st, res, off, N, nres, cap,
                     cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, long_list, nlong, err);
  return hipGetLastError();
}

}  // namespace kd
