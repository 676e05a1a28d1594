// Single-workgroup stable LSD radix sort and block scans.
//
// One workgroup sorts one segment, so a batch of independent segments is
// sorted by a grid with one workgroup per segment.  Keys and values live in
// global memory and ping-pong between two buffers; each pass moves the
// elements in tiles of NT with a wave-level multi-split (ballots on the
// digit bits) so equal digits keep their input order.  A pass whose digit is
// the same for every key is skipped.
#pragma once

#include "kd_internal.h"

namespace kd {

template <int NT>
struct RadixShared {
  static constexpr int NW = NT / 64;
  uint32_t base[256];
  uint32_t tot[256];
  uint32_t wcnt[NW][256];
  uint32_t flag;
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

// Sorts (k0, v0)[0, n) stably by key bits [bit_lo, bit_hi).  Returns 0 when
// the result ends in (k0, v0) and 1 when it ends in (k1, v1).
template <int NT, typename KeyT>
__device__ int block_radix_sort(KeyT *k0, uint32_t *v0, KeyT *k1, uint32_t *v1, uint32_t n,
                                int bit_lo, int bit_hi, RadixShared<NT> &sh) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int cur = 0;
  for (int shift = bit_lo; shift < bit_hi; shift += 8) {
    KeyT *kin = cur ? k1 : k0;
    uint32_t *vin = cur ? v1 : v0;
    KeyT *kout = cur ? k0 : k1;
    uint32_t *vout = cur ? v0 : v1;
    const int nb = (bit_hi - shift) < 8 ? (bit_hi - shift) : 8;
    const uint32_t dmask = (1u << nb) - 1u;
    for (int d = tid; d < 256; d += NT) sh.tot[d] = 0;
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += NT) atomicAdd(&sh.tot[(uint32_t)(kin[i] >> shift) & dmask], 1u);
    __syncthreads();
    for (int d = tid; d < 256; d += NT)
      if (sh.tot[d] == n) sh.flag = 1;
    __syncthreads();
    if (sh.flag) continue;  // identical digit everywhere: the pass is the identity
    if (wave == 0) {
      uint32_t a0 = sh.tot[lane * 4], a1 = sh.tot[lane * 4 + 1];
      uint32_t a2 = sh.tot[lane * 4 + 2], a3 = sh.tot[lane * 4 + 3];
      uint32_t s = a0 + a1 + a2 + a3, incl = s;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      uint32_t ex = incl - s;
      sh.base[lane * 4] = ex;
      sh.base[lane * 4 + 1] = ex + a0;
      sh.base[lane * 4 + 2] = ex + a0 + a1;
      sh.base[lane * 4 + 3] = ex + a0 + a1 + a2;
    }
    for (int x = tid; x < NW * 256; x += NT) (&sh.wcnt[0][0])[x] = 0;
    __syncthreads();
    for (uint32_t t0 = 0; t0 < n; t0 += NT) {
      const uint32_t i = t0 + tid;
      const bool valid = i < n;
      KeyT key = valid ? kin[i] : (KeyT)0;
      uint32_t val = valid ? vin[i] : 0u;
      uint32_t d = valid ? ((uint32_t)(key >> shift) & dmask) : 0u;
      unsigned long long m = __ballot(valid);
      for (int b = 0; b < nb; b++) {
        unsigned long long bb = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bb : ~bb;
      }
      const unsigned long long lt = m & lanemask_lt();
      const uint32_t rank = (uint32_t)__popcll(lt);
      if (valid && lt == 0) sh.wcnt[wave][d] = (uint32_t)__popcll(m);
      __syncthreads();
      for (int d2 = tid; d2 < 256; d2 += NT) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
          uint32_t c = sh.wcnt[w][d2];
          sh.wcnt[w][d2] = run;
          run += c;
        }
        sh.tot[d2] = run;
      }
      __syncthreads();
      if (valid) {
        uint32_t pos = sh.base[d] + sh.wcnt[wave][d] + rank;
        kout[pos] = key;
        vout[pos] = val;
      }
      __syncthreads();
      for (int d2 = tid; d2 < 256; d2 += NT) {
        sh.base[d2] += sh.tot[d2];
#pragma unroll
        for (int w = 0; w < NW; w++) sh.wcnt[w][d2] = 0;
      }
      __syncthreads();
    }
    cur ^= 1;
  }
  return cur;
}

}  // namespace kd
