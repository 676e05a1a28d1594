// k-mer counting (paper Section 3, "k-mer Rank": the count vector c^X of a
// sequence over the epsilon = 6^6 words).
//
// Output per input sequence i, at capacity offset offsets[i] - 5i (the sum
// of K = n - 5 over the sequences before it, so no scan is needed): its
// distinct words in increasing order with their counts, plus D (distinct
// words), K and the number of words seen at least twice.
//
// Sequences of up to 4096 words: one 256-thread workgroup each; the
// residues are mapped through an LDS Dayhoff-6 table and the words
// collected in an LDS presence bitmap (see count_one).  Longer
// sequences (rare) are queued and handled by a persistent kernel that
// histograms into a dense 46656-bin LDS table (two 16-bit bins per word;
// a sequence has at most 65535 words, so a bin never carries).
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

// Counts one sequence of K <= CAP words with one workgroup of NT threads.
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

// First pass, one workgroup per sequence: validates every sequence, counts
// those of at most 1024 words (LDS sized for them), and queues longer ones
// for the 4096-word kernel or the dense-histogram one.
__global__ __launch_bounds__(kCountThreads) void count_short_kernel(
    const uint8_t *__restrict__ res, const uint64_t *__restrict__ off, uint64_t *__restrict__ in_off,
    uint32_t N, uint64_t nres,
    uint64_t cap, uint16_t *__restrict__ cap_ids, uint16_t *__restrict__ cap_cnt,
    uint32_t *__restrict__ hi_cap,
    uint32_t *__restrict__ Dout, uint32_t *__restrict__ Kout, uint32_t *__restrict__ nhiout,
    uint32_t *__restrict__ mid_list, uint32_t *__restrict__ nmid, uint32_t *__restrict__ long_list,
    uint32_t *__restrict__ nlong, unsigned long long *err) {
  constexpr int CAP = 1024;
  __shared__ CountShared<CAP> sh;
  const uint32_t i = blockIdx.x, tid = threadIdx.x;
  for (uint32_t c = tid; c < 256; c += kCountThreads) sh.lut[c] = dayhoff6(c);
  uint64_t o0, o1;
  const uint32_t code = check_offsets(off, i, N, nres, o0, o1);
  if (code != kErrNone) {
    if (tid == 0) atomicMin(err, pack_err(i, code, 0));
    return;
  }
  if (tid == 0) {
    in_off[i] = o0;
    if (i + 1 == N) in_off[N] = o1;
  }
  const uint32_t n = (uint32_t)(o1 - o0);
  const uint32_t K = n - (kK - 1);
  if (K > (uint32_t)CAP) {
    if (tid == 0) {
      if (K <= (uint32_t)kShortMax) mid_list[atomicAdd(nmid, 1u)] = i;
      else long_list[atomicAdd(nlong, 1u)] = i;
    }
    return;
  }
  __syncthreads();
  count_one<CAP>(res, nres, i, o0, n, cap, sh, cap_ids, cap_cnt, hi_cap, Dout, Kout, nhiout, err);
}

// Sequences of 1025..4096 words, queued by the first pass.
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
                        unsigned long long *err, int cus) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(count_short_kernel, dim3(N), dim3(kCountThreads), 0, st, res, off, in_off, N,
                     nres, cap, cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, mid_list, nmid,
                     long_list, nlong, err);
  KD_HIP(hipGetLastError());
  const uint32_t grid = (uint32_t)(cus > 0 ? cus : 256);
  hipLaunchKernelGGL(count_mid_kernel, dim3(2 * grid), dim3(kCountThreads), 0, st, res, off, nres,
                     cap, cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, mid_list, nmid, err);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(count_long_kernel, dim3(grid), dim3(1024), 0, st, res, off, N, nres, cap,
                     cap_ids, cap_cnt, hi_cap, Dorig, Korig, nhi_orig, long_list, nlong, err);
  return hipGetLastError();
}

}  // namespace kd
