// Calibration kernel: the rate of the rank kernel's elementary operation, a
// 16-bit LDS read at a data-dependent (random) index, with K reads of a
// lane issued together before any of their results is used.  It gives the
// ceiling the mask lookups of the all-pairs kernels are measured against.
//
// Each workgroup (1024 threads, as the rank kernel) fills a 64 KB table;
// lane l starts from 32 pseudo-random 15-bit indices and, at step s, reads
// the entries at index ^ m_s (m_s the same 15-bit mask for every lane, so
// each step keeps the random spread of indices over the banks).  The values
// read are folded into one word per lane so nothing is optimized away.
#include "kd_internal.h"

namespace kd {

constexpr uint32_t kProbeEntries = 32768;

template <int K>
__global__ __launch_bounds__(1024) void lds_probe_kernel(uint32_t steps, uint32_t *__restrict__ sink) {
  __shared__ uint16_t T[kProbeEntries];
  const uint32_t tid = threadIdx.x;
  for (uint32_t x = tid; x < kProbeEntries; x += 1024) T[x] = (uint16_t)(x * 40503u);
  uint32_t idx[32];
  uint32_t h = (blockIdx.x * 1024u + tid) * 2654435761u + 0x9E3779B9u;
#pragma unroll
  for (int k = 0; k < 32; k++) {
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    idx[k] = h & (kProbeEntries - 1);
  }
  __syncthreads();
  uint32_t acc = 0;
  for (uint32_t s = 0; s < steps; s++) {
    const uint32_t m = (s * 0x9E37u) & (kProbeEntries - 1);
#pragma unroll
    for (int b = 0; b < 32; b += K) {
      uint32_t v[K];
#pragma unroll
      for (int k = 0; k < K; k++) v[k] = T[idx[b + k] ^ m];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < K; k++) acc = acc * 3u + v[k];
    }
  }
  sink[blockIdx.x * 1024u + tid] = acc;
}

hipError_t launch_lds_probe(hipStream_t st, uint32_t workgroups, uint32_t steps, uint32_t batch,
                            uint32_t *sink) {
  switch (batch) {
    case 2: hipLaunchKernelGGL(lds_probe_kernel<2>, dim3(workgroups), dim3(1024), 0, st, steps, sink); break;
    case 8: hipLaunchKernelGGL(lds_probe_kernel<8>, dim3(workgroups), dim3(1024), 0, st, steps, sink); break;
    case 32: hipLaunchKernelGGL(lds_probe_kernel<32>, dim3(workgroups), dim3(1024), 0, st, steps, sink); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace kd
