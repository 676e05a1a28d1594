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
#include "kd_internal.h"

namespace kd {

// carry-save add: (hi, lo) <- majority / parity of (lo, a, b)
__device__ __forceinline__ void csa(uint32_t &hi, uint32_t &lo, uint32_t a, uint32_t b) {
  const uint32_t u = lo ^ a;
  hi = (u & b) | (~u & lo);
  lo = u ^ b;
}

// Adds 8 words (16 looked-up masks) into the bit planes P (P[k] has weight
// 2^k).  Planes 0-2 are the carry-save state; the weight-8 output ripples
// into planes 3..kmax-1.
__device__ __forceinline__ void add8(uint32_t (&P)[16], const uint32_t (&w)[8], uint32_t kmax) {
  uint32_t twosA, twosB, foursA, foursB, eights;
  csa(twosA, P[0], w[0], w[1]);
  csa(twosB, P[0], w[2], w[3]);
  csa(foursA, P[1], twosA, twosB);
  csa(twosA, P[0], w[4], w[5]);
  csa(twosB, P[0], w[6], w[7]);
  csa(foursB, P[1], twosA, twosB);
  csa(eights, P[2], foursA, foursB);
  uint32_t c = eights;
#pragma unroll
  for (int k = 3; k < 16; k++) {
    if ((uint32_t)k < kmax) {
      const uint32_t t = P[k] & c;
      P[k] ^= c;
      c = t;
    }
  }
}

__device__ __forceinline__ void swap_bits(uint32_t &x, uint32_t &y, int j, uint32_t m) {
  const uint32_t t = ((x >> j) ^ y) & m;
  y ^= t;
  x ^= t << j;
}

// Transposes two 16x16 bit matrices held in the low and high halves of
// A[0..15]: on entry bit (16h + r) of A[k] is bit k of counter (h, r); on
// exit bit (16h + k) of A[r] is that same bit.
__device__ __forceinline__ void transpose16(uint32_t (&A)[16]) {
#pragma unroll
  for (int k = 0; k < 8; k++) swap_bits(A[k], A[k + 8], 8, 0x00FF00FFu);
#pragma unroll
  for (int k = 0; k < 16; k++)
    if (!(k & 4)) swap_bits(A[k], A[k + 4], 4, 0x0F0F0F0Fu);
#pragma unroll
  for (int k = 0; k < 16; k++)
    if (!(k & 2)) swap_bits(A[k], A[k + 2], 2, 0x33333333u);
#pragma unroll
  for (int k = 0; k < 16; k += 2) swap_bits(A[k], A[k + 1], 1, 0x55555555u);
}

__device__ __forceinline__ uint32_t plane_count(uint32_t L) {
  // one-bit counters see at most L/2 words; planes needed = bit length
  const uint32_t h = L >> 1;
  const uint32_t b = 32u - (uint32_t)__clz((int)h);
  return b < 3u ? 3u : (b > 16u ? 16u : b);
}

__device__ __forceinline__ uint32_t look2(const uint16_t *T16, uint32_t x) {
  return (uint32_t)T16[x & 0xFFFFu] | ((uint32_t)T16[x >> 16] << 16);
}

// Level-1 counts of one column (this lane) against the 16 rows of the LDS
// table.  Chunk it (16 words) of the column is at p[2*it*64] and
// p[(2*it+1)*64]; iterations at or beyond niter_lane read sentinel words.
template <bool kUniform>
__device__ __forceinline__ void column_counts(const uint16_t *T16, const uint4 *__restrict__ p,
                                              uint32_t niter_lane, uint32_t niter_wave,
                                              uint32_t kmax, uint32_t (&cnt)[16]) {
  uint32_t P[16];
#pragma unroll
  for (int k = 0; k < 16; k++) P[k] = 0;
  const uint4 sent = make_uint4(0xB640B640u, 0xB640B640u, 0xB640B640u, 0xB640B640u);
  uint4 a = sent, b = sent;
  if (kUniform || niter_lane > 0) {
    a = p[0];
    b = p[64];
  }
  for (uint32_t it = 0; it < niter_wave; it++) {
    uint4 na = sent, nb = sent;
    if (kUniform ? (it + 1 < niter_wave) : (it + 1 < niter_lane)) {
      na = p[(size_t)(2 * it + 2) * 64];
      nb = p[(size_t)(2 * it + 3) * 64];
    }
    uint32_t w[8];
    w[0] = look2(T16, a.x);
    w[1] = look2(T16, a.y);
    w[2] = look2(T16, a.z);
    w[3] = look2(T16, a.w);
    w[4] = look2(T16, b.x);
    w[5] = look2(T16, b.y);
    w[6] = look2(T16, b.z);
    w[7] = look2(T16, b.w);
    add8(P, w, kmax);
    a = na;
    b = nb;
  }
  transpose16(P);
  typedef __attribute__((ext_vector_type(2))) unsigned short us2;
  const us2 ones = __builtin_bit_cast(us2, 0x00010001u);
#pragma unroll
  for (int r = 0; r < 16; r++) cnt[r] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, P[r]), ones, 0u, false);
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

// Reduces 16 values per lane over the 64 lanes with a fixed halving
// butterfly; lanes 4r..4r+3 return the total of value r.
__device__ __forceinline__ double halving_reduce16(const double (&v)[16], uint32_t lane) {
  double u8[8], u4[4], u2[2];
  const bool b5 = lane & 32u, b4 = lane & 16u, b3 = lane & 8u, b2 = lane & 4u;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const double send = b5 ? v[i] : v[i + 8];
    const double keep = b5 ? v[i + 8] : v[i];
    u8[i] = keep + __shfl_xor(send, 32, 64);
  }
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

__device__ __forceinline__ void acc_add(long long *acc, uint32_t s, double x) {
  long long l0, l1, l2;
  fix_limbs(x, l0, l1, l2);
  unsigned long long *a = reinterpret_cast<unsigned long long *>(acc) + 3ull * s;
  atomicAdd(a, (unsigned long long)l0);
  atomicAdd(a + 1, (unsigned long long)l1);
  atomicAdd(a + 2, (unsigned long long)l2);
}

// LDS state of one row block: presence table, count>=2 bitmap, row K.
struct RowShared {
  uint32_t T32[kTableWords];
  uint32_t BM[kBitmapWords];
  uint32_t rowK[16];
};

// Builds the table for rows rowpos(r) (sorted positions; 0xFFFFFFFF = none).
// Requires 1024 threads: wave r inserts row r.
template <class RowPos>
__device__ __forceinline__ void build_rows(const SetView &v, RowPos rowpos,
                                           const uint16_t *__restrict__ exc_ids, uint32_t e0,
                                           uint32_t en, RowShared &sh) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  for (uint32_t x = tid; x < (uint32_t)kTableWords; x += 1024) sh.T32[x] = 0;
  for (uint32_t x = tid; x < (uint32_t)kBitmapWords; x += 1024) sh.BM[x] = 0;
  __syncthreads();
  const uint32_t r = wave, sr = rowpos(r);
  if (sr != 0xFFFFFFFFu) {
    const uint32_t g = sr >> 6, ln = sr & 63u, Dr = v.D[sr];
    const uint16_t *base = v.gids + v.grp_off[g];
    for (uint32_t t = lane; t < Dr; t += 64) {
      const uint32_t id = base[((size_t)(t >> 3) * 64 + ln) * 8 + (t & 7u)];
      atomicOr(&sh.T32[id >> 1], (1u << r) << ((id & 1u) << 4));
    }
    if (lane == 0) sh.rowK[r] = v.K[sr];
  } else if (lane == 0) {
    sh.rowK[r] = 0;
  }
  for (uint32_t e = tid; e < en; e += 1024) {
    const uint32_t id = exc_ids[e0 + e];
    atomicOr(&sh.BM[id >> 5], 1u << (id & 31u));
  }
  __syncthreads();
}

struct ConsecutiveRows {
  uint32_t s0, N;
  __device__ uint32_t operator()(uint32_t r) const { return s0 + r < N ? s0 + r : 0xFFFFFFFFu; }
};

struct ListedRows {
  const uint32_t *pos;
  __device__ uint32_t operator()(uint32_t r) const { return pos[r]; }
};

__global__ __launch_bounds__(1024) void rank_pairs_kernel(const SetView *__restrict__ views,
                                                          const PairTask *__restrict__ tasks,
                                                          double delta) {
  __shared__ RowShared sh;
  const PairTask tk = tasks[blockIdx.x];
  const SetView v = views[tk.set];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t e0 = v.exc_off[tk.rb], en = v.exc_n[tk.rb];
  build_rows(v, ConsecutiveRows{16u * tk.rb, v.N}, v.exc_ids, e0, en, sh);
  const uint16_t *T16 = reinterpret_cast<const uint16_t *>(sh.T32);
  for (uint32_t g = tk.g0 + wave; g < tk.g1; g += 16) {
    const uint32_t sc = 64u * g + lane;
    const bool vc = sc < v.N;
    const uint32_t L = v.grp_len[g];
    const uint4 *p = reinterpret_cast<const uint4 *>(v.gids + v.grp_off[g]) + lane;
    uint32_t cnt[16];
    column_counts<true>(T16, p, L >> 4, L >> 4, plane_count(L), cnt);
    if (vc) column_excess(v, sc, sh.BM, v.exc_ids, v.exc_cnt, e0, en, cnt);
    const uint32_t Kc = vc ? v.K[sc] : 1u;
    double rv[16];
    double colsum = 0.0;
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const uint32_t sr = 16u * tk.rb + r;
      double d = 0.0;
      if (vc && sc < sr && sr < v.N) {
        const uint32_t den = min(sh.rowK[r], Kc);
        d = -log(delta + (double)cnt[r] / (double)den);
      }
      rv[r] = d;
      colsum += d;
    }
    const double rowtot = halving_reduce16(rv, lane);
    if ((lane & 3u) == 0) {
      const uint32_t sr = 16u * tk.rb + (lane >> 2);
      if (sr < v.N) acc_add(v.acc, sr, rowtot);
    }
    if (vc) acc_add(v.acc, sc, colsum);
  }
}

hipError_t launch_rank_pairs(hipStream_t st, const SetView *d_views, const PairTask *tasks,
                             uint32_t ntasks, double delta) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_pairs_kernel, dim3(ntasks), dim3(1024), 0, st, d_views, tasks, delta);
  return hipGetLastError();
}

__global__ void rank_finalize_kernel(SetView v, double delta, double *__restrict__ ranks) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= v.N) return;
  const long long *a = v.acc + 3ull * s;
  long long l0, l1, l2;
  fix_limbs(-log(delta + 1.0), l0, l1, l2);  // the j = i term: F = 1
  const double sum = fix_to_double(a[0] + l0, a[1] + l1, a[2] + l2);
  ranks[v.perm[s]] = sum / (double)v.N;
}

hipError_t launch_rank_finalize(hipStream_t st, const SetView &v, double delta, double *ranks) {
  if (v.N == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_finalize_kernel, dim3((v.N + 255) / 256), dim3(256), 0, st, v, delta,
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
  build_rows(v, ListedRows{rowpos + 16u * bx}, exc_ids, e0, en, sh);
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
  column_counts<false>(T16, p, L >> 4, Lw >> 4, plane_count(Lw), cnt);
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
