// Globalized k-mer rank, the cross pass (paper Section 3.1.1; Algorithm 2
// step 6): every sequence of a counted batch of blocks against the samples
// gathered from all blocks, with the tile machinery of the all-pairs rank
// kernel (tile.h).
#include "tile.h"

namespace kd {

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

}  // namespace kd
