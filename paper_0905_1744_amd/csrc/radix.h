// Single-workgroup stable LSD radix sort and block scans.
//
// One workgroup sorts one segment, so a batch of independent segments is
// sorted by a grid with one workgroup per segment.  Keys and values live in
// global memory and ping-pong between two buffers.  The digit histograms of
// all passes are taken in one read (they do not depend on the order); each
// pass then moves the elements in tiles of 4 x NT with a wave-level
// multi-split (ballots on the digit bits) so equal digits keep their input
// order.  A pass whose digit is the same for every key is skipped; the
// skip decisions of all passes are taken once, right after the histograms,
// and stay read-only while the passes run, so every wave takes the same
// branches and meets the same barriers.
#pragma once

#include "kd_internal.h"

namespace kd {

template <int NT>
struct RadixShared {
  static constexpr int NW = NT / 64;
  static constexpr int SUB = 4;   // elements per thread per tile
  uint32_t hist[8][256];          // digit histograms of every pass
  uint32_t base[256];
  uint32_t tot[256];
  uint16_t wcnt[SUB][NW][256];    // per (sub-tile, wave, digit) counts, then prefixes
  uint32_t skip[8];               // pass q moves nothing (one digit value holds all n keys)
  uint32_t wsum[NW];
};

// Exclusive scan of one value per thread over the workgroup; returns the
// thread's prefix and writes the grand total into `total`.
template <int NT>
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t *wsum, uint32_t &total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; w++) {
    uint32_t s = wsum[w];
    before += (w < wave) ? s : 0;
    all += s;
  }
  __syncthreads();
  total = all;
  return before + incl - x;
}

template <int NT>
__device__ inline unsigned long long block_exclusive_scan64(unsigned long long x,
                                                           unsigned long long *wsum,
                                                           unsigned long long &total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    unsigned long long y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  unsigned long long before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; w++) {
    unsigned long long s = wsum[w];
    before += (w < wave) ? s : 0;
    all += s;
  }
  __syncthreads();
  total = all;
  return before + incl - x;
}

// Sorts (k0, v0)[0, n) stably by key bits [bit_lo, bit_hi) (at most 64
// bits, 8 per pass).  Returns 0 when the result ends in (k0, v0) and 1
// when it ends in (k1, v1).  A tile is SUB x NT elements: element
// t0 + s NT + tid; its position among equal digits of the tile is found
// from ballots (wave), then per-(sub-tile, wave) prefix counts (LDS).
template <int NT, typename KeyT>
__device__ int block_radix_sort(KeyT *k0, uint32_t *v0, KeyT *k1, uint32_t *v1, uint32_t n,
                                int bit_lo, int bit_hi, RadixShared<NT> &sh) {
  constexpr int NW = NT / 64, SUB = RadixShared<NT>::SUB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int npass = (bit_hi - bit_lo + 7) / 8;
  for (int x = tid; x < npass * 256; x += NT) (&sh.hist[0][0])[x] = 0;
  if (tid < 8) sh.skip[tid] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < n; i += NT) {
    const KeyT key = k0[i];
    for (int q = 0; q < npass; q++) {
      const int sh_q = bit_lo + 8 * q, nb_q = (bit_hi - sh_q) < 8 ? (bit_hi - sh_q) : 8;
      atomicAdd(&sh.hist[q][(uint32_t)(key >> sh_q) & ((1u << nb_q) - 1u)], 1u);
    }
  }
  __syncthreads();
  for (int x = tid; x < npass * 256; x += NT)
    if ((&sh.hist[0][0])[x] == n) sh.skip[x >> 8] = 1;
  __syncthreads();
  int cur = 0;
  for (int q = 0; q < npass; q++) {
    const int shift = bit_lo + 8 * q;
    const int nb = (bit_hi - shift) < 8 ? (bit_hi - shift) : 8;
    const uint32_t dmask = (1u << nb) - 1u;
    KeyT *kin = cur ? k1 : k0;
    uint32_t *vin = cur ? v1 : v0;
    KeyT *kout = cur ? k0 : k1;
    uint32_t *vout = cur ? v0 : v1;
    if (sh.skip[q]) continue;  // identical digit everywhere: the pass is the identity
    if (wave == 0) {
      const uint32_t a0 = sh.hist[q][lane * 4], a1 = sh.hist[q][lane * 4 + 1];
      const uint32_t a2 = sh.hist[q][lane * 4 + 2], a3 = sh.hist[q][lane * 4 + 3];
      const uint32_t sum = a0 + a1 + a2 + a3;
      uint32_t incl = sum;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      const uint32_t ex = incl - sum;
      sh.base[lane * 4] = ex;
      sh.base[lane * 4 + 1] = ex + a0;
      sh.base[lane * 4 + 2] = ex + a0 + a1;
      sh.base[lane * 4 + 3] = ex + a0 + a1 + a2;
    }
    for (int x = tid; x < SUB * NW * 256; x += NT) (&sh.wcnt[0][0][0])[x] = 0;
    __syncthreads();
    for (uint32_t t0 = 0; t0 < n; t0 += SUB * NT) {
      KeyT key[SUB];
      uint32_t val[SUB], dig[SUB], rank[SUB];
      bool valid[SUB];
#pragma unroll
      for (int s = 0; s < SUB; s++) {  // issue every load of the tile first
        const uint32_t i = t0 + s * NT + tid;
        valid[s] = i < n;
        key[s] = valid[s] ? kin[i] : (KeyT)0;
        val[s] = valid[s] ? vin[i] : 0u;
      }
#pragma unroll
      for (int s = 0; s < SUB; s++) {
        dig[s] = (uint32_t)(key[s] >> shift) & dmask;
        unsigned long long m = __ballot(valid[s]);
        for (int b = 0; b < nb; b++) {
          const unsigned long long bb = __ballot((dig[s] >> b) & 1u);
          m &= ((dig[s] >> b) & 1u) ? bb : ~bb;
        }
        const unsigned long long lt = m & lanemask_lt();
        rank[s] = (uint32_t)__popcll(lt);
        if (valid[s] && lt == 0) sh.wcnt[s][wave][dig[s]] = (uint16_t)__popcll(m);
      }
      __syncthreads();
      for (int d2 = tid; d2 < 256; d2 += NT) {
        uint32_t run = 0;
        for (int s = 0; s < SUB; s++)
#pragma unroll
          for (int w = 0; w < NW; w++) {
            const uint32_t c = sh.wcnt[s][w][d2];
            sh.wcnt[s][w][d2] = (uint16_t)run;
            run += c;
          }
        sh.tot[d2] = run;
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < SUB; s++) {
        if (valid[s]) {
          const uint32_t pos = sh.base[dig[s]] + sh.wcnt[s][wave][dig[s]] + rank[s];
          kout[pos] = key[s];
          vout[pos] = val[s];
        }
      }
      __syncthreads();
      for (int d2 = tid; d2 < 256; d2 += NT) {
        sh.base[d2] += sh.tot[d2];
        for (int s = 0; s < SUB; s++)
#pragma unroll
          for (int w = 0; w < NW; w++) sh.wcnt[s][w][d2] = 0;
      }
      __syncthreads();
    }
    cur ^= 1;
  }
  return cur;
}

}  // namespace kd
