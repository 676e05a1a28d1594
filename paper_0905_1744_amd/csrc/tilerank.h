// Rank of every key of an array among all keys, for keys made unique by
// their index: rank(i) = #{j : (key_j, j) < (key_i, i)}, i.e. the position
// of i in the stably sorted order.
//
// Two kernels.  tile_sort: each workgroup sorts one tile of kTileKeys
// (key, index) pairs in LDS with a bitonic network and stores the sorted
// tile (and zeroes the ranks of its keys).  tile_count: workgroup (c, t)
// stages sorted tile t in LDS and adds, for each of its 1024 keys i, the
// number of pairs of tile t below (key_i, i) -- a binary search -- to
// rank(i).  Work is n log(kTileKeys) per tile instead of n per key.
#pragma once

#include "kd_internal.h"

namespace kd {

constexpr uint32_t kTileKeys = 512;
constexpr uint32_t kTileSortThreads = 256;

struct KeyIdx {
  unsigned long long k;
  uint32_t i;
  uint32_t pad;
};

__device__ __forceinline__ bool key_less(const KeyIdx &a, const KeyIdx &b) {
  return a.k < b.k || (a.k == b.k && a.i < b.i);
}

template <class KeyFn>
__global__ __launch_bounds__(kTileSortThreads) void tile_sort_kernel(KeyFn key, uint32_t n,
                                                         KeyIdx *__restrict__ sorted,
                                                         uint32_t *__restrict__ rank) {
  __shared__ KeyIdx sk[kTileKeys];
  const uint32_t t0 = blockIdx.x * kTileKeys, tid = threadIdx.x;
  const uint32_t m = min(kTileKeys, n - t0);
  uint32_t P = 2;
  while (P < m) P <<= 1;
  for (uint32_t x = tid; x < P; x += kTileSortThreads) {
    KeyIdx v;
    v.k = x < m ? key(t0 + x) : ~0ull;
    v.i = x < m ? t0 + x : 0xFFFFFFFFu;
    v.pad = 0;
    sk[x] = v;
    if (x < m) rank[t0 + x] = 0;
  }
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t x = tid; x < (P >> 1); x += kTileSortThreads) {
        const uint32_t a = ((x & ~(j - 1)) << 1) | (x & (j - 1));
        const uint32_t b = a | j;
        const KeyIdx va = sk[a], vb = sk[b];
        if (key_less(vb, va) == ((a & k) == 0)) {
          sk[a] = vb;
          sk[b] = va;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t x = tid; x < m; x += kTileSortThreads) sorted[t0 + x] = sk[x];
}

template <class KeyFn>
__global__ __launch_bounds__(1024) void tile_count_kernel(KeyFn key, uint32_t n,
                                                         const KeyIdx *__restrict__ sorted,
                                                         uint32_t *__restrict__ rank) {
  __shared__ KeyIdx sk[kTileKeys];
  const uint32_t t0 = blockIdx.y * kTileKeys, m = min(kTileKeys, n - t0);
  for (uint32_t x = threadIdx.x; x < m; x += 1024) sk[x] = sorted[t0 + x];
  __syncthreads();
  const uint32_t i = blockIdx.x * 1024u + threadIdx.x;
  if (i >= n) return;
  KeyIdx q;
  q.k = key(i);
  q.i = i;
  uint32_t lo = 0, hi = m;  // first element not below q
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (key_less(sk[mid], q)) lo = mid + 1;
    else hi = mid;
  }
  if (lo) atomicAdd(&rank[i], lo);
}

// rank[0..n) as defined above; sorted needs n entries of scratch
template <class KeyFn>
hipError_t launch_tile_rank(hipStream_t st, KeyFn key, uint32_t n, KeyIdx *sorted, uint32_t *rank) {
  if (n == 0) return hipSuccess;
  const uint32_t T = (n + kTileKeys - 1) / kTileKeys;
  hipLaunchKernelGGL(tile_sort_kernel<KeyFn>, dim3(T), dim3(kTileSortThreads), 0, st, key, n, sorted,
                     rank);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(tile_count_kernel<KeyFn>, dim3((n + 1023) / 1024, T), dim3(1024), 0, st, key, n,
                     sorted, rank);
  return hipGetLastError();
}

}  // namespace kd
