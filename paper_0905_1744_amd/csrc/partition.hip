// Regular-sampling decomposition (paper Section 3.1.2; Algorithm 2 steps 3
// and 8-11) with B virtual processors on one GPU.
//
// One workgroup handles one set (a batch of sets runs one workgroup per set):
//  1. keys (rank, index) are sorted once (stable LSD radix sort of an
//     order-preserving 64-bit image of the rank over index-ordered input);
//     the sorted indices are the grouped output order and give every key its
//     global position rho, so later key comparisons are integer compares;
//  2. a stable counting sort of that order by virtual block (block b holds
//     input indices [floor(bn/B), floor((b+1)n/B))) yields each block in key
//     order, i.e. the paper's local sorts;
//  3. block b contributes the keys at 0-based local positions
//     floor(t w_b / B), t = 1..B-1, as regular samples;
//  4. the B(B-1) samples are sorted (by rho) and the ones at 0-based
//     positions (i-1)B + floor(B/2) - 1, i = 1..B-1, become the pivots;
//  5. bucket = number of pivots with smaller rho; bucket b starts at
//     rho(pivot_{b-1}) + 1 in the key order.
//
// A single set takes a fully parallel route instead (up to 8192 samples):
// rho_i = #{j : (R_j, j) < (R_i, i)} comes from ranking against sorted
// tiles of keys (tilerank.h); ranking the keys (block(i), rho_i) the same
// way gives each key its slot in the concatenation of the locally sorted
// blocks; samples / pivots / buckets then follow from rho exactly as above.
#include "radix.h"
#include "tilerank.h"

namespace kd {


__device__ __forceinline__ unsigned long long rank_key(double r) {
  if (r == 0.0) r = 0.0;  // -0 and +0 are the same rank
  const unsigned long long b = (unsigned long long)__double_as_longlong(r);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

__device__ __forceinline__ uint32_t bitlen(uint32_t x) { return x ? 32u - (uint32_t)__clz((int)x) : 0u; }

struct PartScratch {
  unsigned long long *k0, *k1;
  uint32_t *v0, *v1, *bk0, *bk1, *bv0, *bv1, *rho;
  uint32_t *sk0, *sk1, *sv0, *sv1, *prho;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline PartScratch carve(void *base, uint32_t n, uint32_t B) {
  PartScratch s;
  char *p = (char *)base;
  const size_t S = (size_t)B * (B - 1);
  s.k0 = (unsigned long long *)p; p += align256(8ull * n);
  s.k1 = (unsigned long long *)p; p += align256(8ull * n);
  uint32_t **u[] = {&s.v0, &s.v1, &s.bk0, &s.bk1, &s.bv0, &s.bv1, &s.rho};
  for (uint32_t **q : u) { *q = (uint32_t *)p; p += align256(4ull * n); }
  uint32_t **w[] = {&s.sk0, &s.sk1, &s.sv0, &s.sv1};
  for (uint32_t **q : w) { *q = (uint32_t *)p; p += align256(4ull * (S ? S : 1)); }
  s.prho = (uint32_t *)p;
  return s;
}

size_t partition_scratch_bytes(uint32_t n, uint32_t B) {
  const size_t S = (size_t)B * (B - 1);
  return 2 * align256(8ull * n) + 7 * align256(4ull * n) + 4 * align256(4ull * (S ? S : 1)) +
         align256(4ull * B) + 256;
}

// One set with a workgroup of NT threads.
template <int NT>
__device__ void partition_one(const double *__restrict__ R, uint32_t n, uint32_t B,
                              uint32_t *__restrict__ bucket, uint32_t *__restrict__ order,
                              uint32_t *__restrict__ offsets, double *__restrict__ piv_r,
                              uint32_t *__restrict__ piv_i, PartScratch s, RadixShared<NT> &sh,
                              uint32_t *s_prho) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < n; i += NT) {
    s.k0[i] = rank_key(R[i]);
    s.v0[i] = i;
  }
  __syncthreads();
  // 1. global key order
  const int w1 = block_radix_sort<NT, unsigned long long>(s.k0, s.v0, s.k1, s.v1, n, 0, 64, sh);
  const uint32_t *vs = w1 ? s.v1 : s.v0;
  for (uint32_t p = tid; p < n; p += NT) {
    const uint32_t idx = vs[p];
    order[p] = idx;
    s.rho[idx] = p;
    // virtual block of idx: largest b with floor(b n / B) <= idx
    s.bk0[p] = (uint32_t)(((unsigned long long)(idx + 1) * B - 1) / n);
    s.bv0[p] = idx;
  }
  __syncthreads();
  // 2. local sorts: stable split of the key order by block
  const int w2 = block_radix_sort<NT, uint32_t>(s.bk0, s.bv0, s.bk1, s.bv1, n, 0, (int)bitlen(B - 1), sh);
  const uint32_t *bs = w2 ? s.bv1 : s.bv0;
  // 3. regular samples
  const uint32_t S = B * (B - 1);
  for (uint32_t q = tid; q < S; q += NT) {
    const uint32_t b = q / (B - 1), t = q % (B - 1) + 1;
    const uint32_t lo = (uint32_t)((unsigned long long)b * n / B);
    const uint32_t w = (uint32_t)((unsigned long long)(b + 1) * n / B) - lo;
    const uint32_t idx = bs[lo + (uint32_t)((unsigned long long)t * w / B)];
    s.sk0[q] = s.rho[idx];
    s.sv0[q] = idx;
  }
  __syncthreads();
  // 4. pivots
  const int w3 = block_radix_sort<NT, uint32_t>(s.sk0, s.sv0, s.sk1, s.sv1, S, 0, (int)bitlen(n - 1), sh);
  const uint32_t *ss = w3 ? s.sk1 : s.sk0;
  const uint32_t *sv = w3 ? s.sv1 : s.sv0;
  for (uint32_t i = tid; i + 1 < B; i += NT) {
    const uint32_t pos = i * B + B / 2 - 1;
    s_prho[i] = ss[pos];
    if (piv_i) piv_i[i] = sv[pos];
    if (piv_r) piv_r[i] = R[sv[pos]];
    offsets[i + 1] = ss[pos] + 1;
  }
  if (tid == 0) {
    offsets[0] = 0;
    offsets[B] = n;
  }
  __syncthreads();
  // 5. buckets
  for (uint32_t i = tid; i < n; i += NT) {
    const uint32_t r = s.rho[i];
    uint32_t lo = 0, hi = B - 1;  // count pivots with prho < r
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_prho[mid] < r) lo = mid + 1;
      else hi = mid;
    }
    bucket[i] = lo;
  }
}

__global__ __launch_bounds__(1024) void partition_kernel(const double *R, uint32_t n, uint32_t B,
                                                         uint32_t *bucket, uint32_t *order,
                                                         uint32_t *offsets, double *piv_r,
                                                         uint32_t *piv_i, void *scratch) {
  __shared__ RadixShared<1024> sh;
  __shared__ uint32_t prho[kMaxBuckets];
  partition_one<1024>(R, n, B, bucket, order, offsets, piv_r, piv_i, carve(scratch, n, B), sh, prho);
}

template <int NT>
__global__ __launch_bounds__(NT) void partition_batch_kernel(const PartDesc *__restrict__ desc,
                                                             const double *R, uint32_t *bucket,
                                                             uint32_t *order, uint32_t *offsets,
                                                             double *piv_r, uint32_t *piv_i,
                                                             char *scratch) {
  __shared__ RadixShared<NT> sh;
  __shared__ uint32_t prho[kMaxBuckets];
  const PartDesc d = desc[blockIdx.x];
  partition_one<NT>(R + d.first, d.n, d.B, bucket + d.first, order + d.first, offsets + d.off_base,
                    piv_r ? piv_r + d.piv_base : nullptr, piv_i ? piv_i + d.piv_base : nullptr,
                    carve(scratch + d.scratch_off, d.n, d.B), sh, prho);
}

// A set's sorts are a chain of passes and barriers, so a batch of small
// sets runs faster with small workgroups, several sets per compute unit at
// once (LDS ~18 KB per 256-thread workgroup against ~42 KB per 1,024).
constexpr uint32_t kSmallPartition = 4096;  // keys or samples per set

hipError_t launch_partition_batch(hipStream_t st, const PartDesc *desc, uint32_t nsets,
                                  uint32_t max_keys, const double *ranks, uint32_t *bucket,
                                  uint32_t *order, uint32_t *offsets, double *pivot_rank,
                                  uint32_t *pivot_idx, void *scratch) {
  if (nsets == 0) return hipSuccess;
  if (max_keys <= kSmallPartition)
    hipLaunchKernelGGL(partition_batch_kernel<256>, dim3(nsets), dim3(256), 0, st, desc, ranks, bucket,
                       order, offsets, pivot_rank, pivot_idx, (char *)scratch);
  else
    hipLaunchKernelGGL(partition_batch_kernel<1024>, dim3(nsets), dim3(1024), 0, st, desc, ranks, bucket,
                       order, offsets, pivot_rank, pivot_idx, (char *)scratch);
  return hipGetLastError();
}

struct RankKeyOf {  // order-preserving image of the rank
  const double *R;
  __device__ unsigned long long operator()(uint32_t i) const { return rank_key(R[i]); }
};

struct BlockRhoOf {  // (virtual block, rho): the locally sorted blocks, concatenated
  const uint32_t *rho;
  uint32_t n, B;
  __device__ unsigned long long operator()(uint32_t i) const {
    const uint32_t b = (uint32_t)(((unsigned long long)(i + 1) * B - 1) / n);
    return ((unsigned long long)b << 32) | rho[i];
  }
};

// order[rho_i] = i (the key order); loc[slot_i] = i (block by block, each
// in key order); with a single block loc is the key order itself.
__global__ __launch_bounds__(256) void scatter_order_kernel(uint32_t n, const uint32_t *__restrict__ rho,
                                                            const uint32_t *__restrict__ slot,
                                                            uint32_t *__restrict__ order,
                                                            uint32_t *__restrict__ loc) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  order[rho[i]] = i;
  if (slot) loc[slot[i]] = i;
}

// Samples, their order, and the pivots / offsets (one workgroup).  The
// B(B-1) sample positions are sorted by rho with a bitonic network in LDS.
constexpr uint32_t kBitonicSamples = 8192;

__global__ __launch_bounds__(1024) void pivots_kernel(const double *__restrict__ R, uint32_t n,
                                                      uint32_t B, const uint32_t *__restrict__ rho,
                                                      const uint32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ loc,
                                                      uint32_t *__restrict__ prho_out,
                                                      uint32_t *__restrict__ offsets,
                                                      double *__restrict__ piv_r,
                                                      uint32_t *__restrict__ piv_i) {
  __shared__ uint32_t smp[kBitonicSamples];
  const uint32_t tid = threadIdx.x;
  const uint32_t S = B * (B - 1);
  uint32_t P = 1;
  while (P < S) P <<= 1;
  for (uint32_t q = tid; q < P; q += 1024) {
    uint32_t v = 0xFFFFFFFFu;
    if (q < S) {
      const uint32_t b = q / (B - 1), t = q % (B - 1) + 1;
      const uint32_t lo = (uint32_t)((unsigned long long)b * n / B);
      const uint32_t w = (uint32_t)((unsigned long long)(b + 1) * n / B) - lo;
      v = rho[loc[lo + (uint32_t)((unsigned long long)t * w / B)]];
    }
    smp[q] = v;
  }
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t x = tid; x < (P >> 1); x += 1024) {
        const uint32_t a = ((x & ~(j - 1)) << 1) | (x & (j - 1));
        const uint32_t b = a | j;
        const uint32_t va = smp[a], vb = smp[b];
        if ((va > vb) == ((a & k) == 0)) {
          smp[a] = vb;
          smp[b] = va;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = tid; i + 1 < B; i += 1024) {
    const uint32_t r = smp[i * B + B / 2 - 1];
    prho_out[i] = r;
    offsets[i + 1] = r + 1;
    const uint32_t idx = order[r];
    if (piv_i) piv_i[i] = idx;
    if (piv_r) piv_r[i] = R[idx];
  }
  if (tid == 0) {
    offsets[0] = 0;
    offsets[B] = n;
  }
}

__global__ __launch_bounds__(256) void bucket_kernel(uint32_t n, uint32_t B,
                                                     const uint32_t *__restrict__ rho,
                                                     const uint32_t *__restrict__ prho,
                                                     uint32_t *__restrict__ bucket) {
  __shared__ uint32_t sp[kMaxBuckets];
  for (uint32_t q = threadIdx.x; q + 1 < B; q += 256) sp[q] = prho[q];
  __syncthreads();
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const uint32_t r = rho[i];
  uint32_t lo = 0, hi = B - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sp[mid] < r) lo = mid + 1;
    else hi = mid;
  }
  bucket[i] = lo;
}

hipError_t launch_partition(hipStream_t st, const double *ranks, uint32_t n, uint32_t B,
                            uint32_t *bucket, uint32_t *order, uint32_t *offsets,
                            double *pivot_rank, uint32_t *pivot_idx, void *scratch) {
  const uint64_t S = (uint64_t)B * (B - 1);
  if (S > kBitonicSamples) {
    hipLaunchKernelGGL(partition_kernel, dim3(1), dim3(1024), 0, st, ranks, n, B, bucket, order,
                       offsets, pivot_rank, pivot_idx, scratch);
    return hipGetLastError();
  }
  char *p = static_cast<char *>(scratch);
  KeyIdx *sorted = reinterpret_cast<KeyIdx *>(p);
  p += align256(sizeof(KeyIdx) * n);
  uint32_t *rho = reinterpret_cast<uint32_t *>(p);
  p += align256(4ull * n);
  uint32_t *slot = reinterpret_cast<uint32_t *>(p);
  p += align256(4ull * n);
  uint32_t *loc = reinterpret_cast<uint32_t *>(p);
  p += align256(4ull * n);
  uint32_t *prho = reinterpret_cast<uint32_t *>(p);
  KD_HIP(launch_tile_rank(st, RankKeyOf{ranks}, n, sorted, rho));
  if (B > 1) KD_HIP(launch_tile_rank(st, BlockRhoOf{rho, n, B}, n, sorted, slot));
  const uint32_t gi = (n + 255) / 256;
  hipLaunchKernelGGL(scatter_order_kernel, dim3(gi), dim3(256), 0, st, n, rho,
                     B > 1 ? slot : nullptr, order, loc);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(pivots_kernel, dim3(1), dim3(1024), 0, st, ranks, n, B, rho, order,
                     B > 1 ? loc : order, prho, offsets, pivot_rank, pivot_idx);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(bucket_kernel, dim3(gi), dim3(256), 0, st, n, B, rho, prho, bucket);
  return hipGetLastError();
}

}  // namespace kd
