// Device layout of a counted set.
//
// Sequences are re-ordered by ascending number of distinct words D (ties by
// input index).  In that order:
//  * column groups of 64 consecutive sequences store their distinct words
//    interleaved (lane l = sequence 64g + l; 8 words per lane per 16-byte
//    chunk; chunks of the 64 lanes adjacent), each list padded with a
//    sentinel word up to the group's longest list rounded to 16, so one
//    wave reads 64 lists with fully coalesced 16-byte loads;
//  * entries with count >= 2 are kept in a separate short CSR list;
//  * every row block of 16 sequences gets the merged, sorted set of words
//    that some row of the block holds at least twice, with the 16 counts.
#include "radix.h"

namespace kd {

// One workgroup per set: stable radix sort of the set's keys with their
// local indices as values.
__global__ __launch_bounds__(1024) void sort_u32_index_kernel(const uint32_t *__restrict__ keys,
                                                              const uint32_t *__restrict__ seq,
                                                              int bits,
                                                              uint32_t *__restrict__ perm,
                                                              uint32_t *k0, uint32_t *v0,
                                                              uint32_t *k1, uint32_t *v1) {
  __shared__ RadixShared<1024> sh;
  const uint32_t a = seq[blockIdx.x], N = seq[blockIdx.x + 1] - a;
  if (N == 0) return;
  keys += a;
  perm += a;
  k0 += a;
  v0 += a;
  k1 += a;
  v1 += a;
  for (uint32_t i = threadIdx.x; i < N; i += 1024) {
    k0[i] = keys[i];
    v0[i] = i;
  }
  __syncthreads();
  const int where = block_radix_sort<1024, uint32_t>(k0, v0, k1, v1, N, 0, bits, sh);
  const uint32_t *src = where ? v1 : v0;
  for (uint32_t i = threadIdx.x; i < N; i += 1024) perm[i] = src[i];
}

hipError_t launch_sort_u32_index(hipStream_t st, const uint32_t *keys, const Segs &sg, uint32_t N,
                                 int bits, uint32_t *perm, uint32_t *scratch_keys,
                                 uint32_t *scratch_vals) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(sort_u32_index_kernel, dim3(sg.nsets), dim3(1024), 0, st, keys, sg.seq, bits,
                     perm, scratch_keys, scratch_vals, scratch_keys + N, scratch_vals + N);
  return hipGetLastError();
}

// Per sorted position: inverse permutation, K, 1/K, D and the count of
// entries seen at least twice (into hcount).  perm and inv hold indices
// local to the set.
__global__ void layout_gather_kernel(Segs sg, uint32_t N, const uint32_t *__restrict__ perm,
                                     const uint32_t *__restrict__ Dorig,
                                     const uint32_t *__restrict__ Korig,
                                     const uint32_t *__restrict__ nhi_orig,
                                     uint32_t *__restrict__ inv, uint32_t *__restrict__ K,
                                     uint32_t *__restrict__ D, double *__restrict__ invK,
                                     uint32_t *__restrict__ hcount, const unsigned long long *err) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N || *err != ~0ull) return;
  const uint32_t a = sg.seq[seg_of(sg.seq, sg.nsets, s)];
  const uint32_t i = a + perm[s];
  inv[i] = s - a;
  K[s] = Korig[i];
  invK[s] = 1.0 / (double)Korig[i];
  D[s] = Dorig[i];
  hcount[s] = nhi_orig[i];
}

// Exclusive scan of n values with one 1024-thread workgroup, each thread
// summing a contiguous chunk; out[n] gets the total, which is returned.
template <typename In, typename Out>
__device__ Out chunked_scan(const In &in, uint32_t n, Out *out, Out *wsum) {
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (n + 1023) / 1024;
  const uint32_t lo = min(tid * per, n), hi = min(lo + per, n);
  Out local = 0;
  for (uint32_t x = lo; x < hi; x++) local += in(x);
  const int lane = tid & 63, wave = tid >> 6;
  Out incl = local;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const Out y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  Out before = 0, all = 0;
  for (int w = 0; w < 16; w++) {
    before += (w < wave) ? wsum[w] : 0;
    all += wsum[w];
  }
  __syncthreads();
  Out run = before + incl - local;
  for (uint32_t x = lo; x < hi; x++) {
    out[x] = run;
    run += in(x);
  }
  if (tid == 0) out[n] = all;
  return all;
}

struct HcountIn {
  const uint32_t *h;
  __device__ uint32_t operator()(uint32_t s) const { return h[s]; }
};
struct GroupIn {
  const uint32_t *len;
  __device__ unsigned long long operator()(uint32_t g) const { return 64ull * len[g]; }
};
// count>=2 entries of the 16 rows of batch-wide row block x
struct BlockHiIn {
  Segs sg;
  const uint32_t *hi_off;
  __device__ uint32_t operator()(uint32_t x) const {
    const uint32_t s = seg_of(sg.rb, sg.nsets, x);
    const uint32_t a = sg.seq[s], n = sg.seq[s + 1] - a, rb = x - sg.rb[s];
    return hi_off[a + min(16u * rb + 16u, n)] - hi_off[a + 16u * rb];
  }
};

__global__ __launch_bounds__(1024) void layout_meta_kernel(
    Segs sg, uint32_t N, uint32_t G, uint32_t RB, const uint32_t *__restrict__ D,
    const uint32_t *__restrict__ hcount, uint32_t *__restrict__ hi_off,
    uint64_t *__restrict__ grp_off, uint32_t *__restrict__ grp_len,
    uint64_t *__restrict__ ghi_off, uint32_t *__restrict__ ghi_len,
    uint32_t *__restrict__ exc_off, const unsigned long long *err, LayoutMeta *meta) {
  __shared__ uint32_t wsum[16];
  __shared__ unsigned long long wsum64[16];
  __shared__ unsigned long long s_ent[16];
  __shared__ uint32_t s_max[16];
  const uint32_t tid = threadIdx.x;
  if (*err != ~0ull) {  // counting failed: report only the error
    if (tid == 0) {
      meta->err = *err;
      meta->n_hi = meta->n_gids = meta->n_exc = meta->entries = meta->max_len = meta->n_ghi = 0;
    }
    return;
  }
  const uint32_t n_hi = chunked_scan(HcountIn{hcount}, N, hi_off, wsum);
  // column group x of set s holds positions a + 64 g .. (g = x - grp[s]);
  // padded length = longest list (the last one: D ascending) rounded to 16;
  // count>=2 entries: longest lane, rounded up to 4
  uint32_t mx = 0;
  for (uint32_t x = tid; x < G; x += 1024) {
    const uint32_t s = seg_of(sg.grp, sg.nsets, x);
    const uint32_t a = sg.seq[s], n = sg.seq[s + 1] - a, g = x - sg.grp[s];
    const uint32_t p0 = a + 64u * g, p1 = a + min(64u * g + 64u, n);
    const uint32_t L = (D[p1 - 1] + 15u) & ~15u;
    grp_len[x] = L;
    mx = max(mx, L);
    uint32_t m = 0;
    for (uint32_t p = p0; p < p1; p++) m = max(m, hcount[p]);
    ghi_len[x] = (m + 3u) & ~3u;
  }
#pragma unroll
  for (int o = 32; o; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
  if ((tid & 63) == 0) s_max[tid >> 6] = mx;
  __syncthreads();
  const unsigned long long n_gids = chunked_scan(GroupIn{grp_len}, G, (unsigned long long *)grp_off, wsum64);
  const unsigned long long n_ghi = chunked_scan(GroupIn{ghi_len}, G, (unsigned long long *)ghi_off, wsum64);
  const uint32_t n_exc = chunked_scan(BlockHiIn{sg, hi_off}, RB, exc_off, wsum);
  unsigned long long ent = 0;
  for (uint32_t s = tid; s < N; s += 1024) ent += D[s];
#pragma unroll
  for (int o = 32; o; o >>= 1) ent += __shfl_xor(ent, o, 64);
  if ((tid & 63) == 0) s_ent[tid >> 6] = ent;
  __syncthreads();
  if (tid == 0) {
    unsigned long long e = 0;
    uint32_t m = 0;
    for (int w = 0; w < 16; w++) {
      e += s_ent[w];
      m = max(m, s_max[w]);
    }
    meta->err = ~0ull;
    meta->n_hi = n_hi;
    meta->n_gids = n_gids;
    meta->n_exc = n_exc;
    meta->entries = e;
    meta->max_len = m;
    meta->n_ghi = n_ghi;
  }
}

hipError_t launch_layout_meta(hipStream_t st, const Segs &sg, uint32_t N, uint32_t G,
                              uint32_t RB, const uint32_t *perm,
                              const uint32_t *Dorig, const uint32_t *Korig,
                              const uint32_t *nhi_orig, uint32_t *inv, uint32_t *K, uint32_t *D,
                              double *invK, uint32_t *hcount, uint32_t *hi_off, uint64_t *grp_off,
                              uint32_t *grp_len, uint64_t *ghi_off, uint32_t *ghi_len,
                              uint32_t *exc_off, const unsigned long long *err, LayoutMeta *meta) {
  hipLaunchKernelGGL(layout_gather_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sg, N, perm,
                     Dorig, Korig, nhi_orig, inv, K, D, invK, hcount, err);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(layout_meta_kernel, dim3(1), dim3(1024), 0, st, sg, N, G, RB, D, hcount,
                     hi_off, grp_off, grp_len, ghi_off, ghi_len, exc_off, err, meta);
  return hipGetLastError();
}

// Grid (batch-wide column group, slice of 16 chunks), 256 threads: lane
// l = tid % 64 writes chunks 16 y + tid / 64 + 4 k (k = 0..3) of sequence
// 64 g + l of the group's set into the interleaved layout (the 64 lanes'
// 16-byte chunks adjacent).
__global__ __launch_bounds__(256) void layout_groups_kernel(Segs sg,
                                                            const uint64_t *__restrict__ offsets,
                                                            const uint16_t *__restrict__ cap_ids,
                                                            uint16_t *__restrict__ gids) {
  const uint32_t x = blockIdx.x, lane = threadIdx.x & 63u, sub = threadIdx.x >> 6;
  const uint32_t set = seg_of(sg.grp, sg.nsets, x);
  const SetView &v = sg.views[set];
  const uint32_t g = x - sg.grp[set];
  const uint32_t L = v.grp_len[g];
  const uint32_t t8_0 = blockIdx.y * 16u;
  if (t8_0 * 8u >= L) return;
  const uint32_t s = 64u * g + lane;
  uint32_t Dl = 0;
  const uint16_t *src = nullptr;
  if (s < v.N) {
    const uint32_t i = v.base + v.perm[s];
    src = cap_ids + (offsets[i] - 5ull * i);
    Dl = v.D[s];
  }
  uint4 *dst = reinterpret_cast<uint4 *>(gids + v.grp_off[g]) + lane;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t t8 = t8_0 + sub + 4u * k;
    if (t8 * 8u >= L) break;
    uint32_t e[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const uint32_t t = t8 * 8 + u;
      e[u] = t < Dl ? src[t] : kSentinel;
    }
    uint4 q;
    q.x = e[0] | (e[1] << 16);
    q.y = e[2] | (e[3] << 16);
    q.z = e[4] | (e[5] << 16);
    q.w = e[6] | (e[7] << 16);
    dst[(size_t)t8 * 64] = q;
  }
}

// One wave per batch-wide sorted position: entries with count >= 2,
// compacted in order.
__global__ __launch_bounds__(256) void layout_hi_kernel(Segs sg, uint32_t N,
                                                        const uint64_t *__restrict__ offsets,
                                                        const uint16_t *__restrict__ cap_ids,
                                                        const uint16_t *__restrict__ cap_cnt,
                                                        uint16_t *__restrict__ hi_ids,
                                                        uint16_t *__restrict__ hi_cnt,
                                                        uint32_t *__restrict__ ghi) {
  const uint32_t p = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (p >= N) return;
  const uint32_t set = seg_of(sg.seq, sg.nsets, p);
  const SetView &v = sg.views[set];
  const uint32_t s = p - v.base;
  const uint32_t i = v.base + v.perm[s];
  const uint64_t co = offsets[i] - 5ull * i;
  const uint32_t Dl = v.D[s];
  const uint32_t h0 = v.hi_off[s];
  const uint64_t gb = v.ghi_off[s >> 6];
  uint32_t o = h0;
  for (uint32_t b = 0; b < Dl; b += 64) {
    const uint32_t t = b + lane;
    uint16_t id = 0, c = 0;
    if (t < Dl) {
      id = cap_ids[co + t];
      c = cap_cnt[co + t];
    }
    const bool f = t < Dl && c >= 2;
    const unsigned long long m = __ballot(f);
    if (f) {
      const uint32_t q = o + (uint32_t)__popcll(m & lanemask_lt());
      hi_ids[q] = id;
      hi_cnt[q] = c;
      ghi[gb + 64ull * (q - h0) + (s & 63u)] = (uint32_t)id | ((uint32_t)c << 16);
    }
    o += (uint32_t)__popcll(m);
  }
}

hipError_t launch_layout_fill(hipStream_t st, const Segs &sg, const SetView &v,
                              const uint64_t *offsets,
                              const uint16_t *cap_ids, const uint16_t *cap_cnt, uint16_t *gids,
                              uint16_t *hi_ids, uint16_t *hi_cnt, uint32_t *ghi,
                              uint32_t max_len) {
  if (v.N == 0) return hipSuccess;
  const uint32_t slices = (max_len / 8 + 15) / 16;
  hipLaunchKernelGGL(layout_groups_kernel, dim3(v.G, slices > 0 ? slices : 1), dim3(256), 0, st, sg,
                     offsets, cap_ids, gids);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(layout_hi_kernel, dim3((v.N + 3) / 4), dim3(256), 0, st, sg, v.N, offsets,
                     cap_ids, cap_cnt, hi_ids, hi_cnt, ghi);
  return hipGetLastError();
}

// Merged count>=2 words of row blocks.  A quarter-wave (16 lanes, one per
// row) merges one block: each lane walks its row's sorted list, the quarter
// agrees on the smallest pending word, and every lane writes its row's
// count for it (0 when the row lacks it).
__global__ __launch_bounds__(64) void exc_build_kernel(Segs sg, uint32_t nblocks,
                                                        const uint32_t *__restrict__ rowpos,
                                                        const uint32_t *__restrict__ exc_off,
                                                        uint32_t *__restrict__ exc_n,
                                                        uint16_t *__restrict__ exc_ids,
                                                        uint16_t *__restrict__ exc_cnt) {
  const uint32_t gq = blockIdx.x * 4 + (threadIdx.x >> 4);  // block handled by this quarter
  const uint32_t r = threadIdx.x & 15;
  const bool active = gq < nblocks;
  uint32_t s = 0xFFFFFFFFu;
  uint32_t set = 0;
  if (active) {
    if (rowpos) {
      s = rowpos[16u * gq + r];
    } else {
      set = seg_of(sg.rb, sg.nsets, gq);
      const uint32_t rb = gq - sg.rb[set];
      if (16u * rb + r < sg.seq[set + 1] - sg.seq[set]) s = 16u * rb + r;
    }
  }
  const SetView &v = sg.views[set];
  uint32_t p = 0, pe = 0;
  if (s != 0xFFFFFFFFu) {
    p = v.hi_off[s];
    pe = v.hi_off[s + 1];
  }
  const uint32_t base = active ? exc_off[gq] : 0;
  uint32_t e = 0;
  while (true) {
    uint32_t cur = p < pe ? v.hi_ids[p] : 0xFFFFFFFFu;
    uint32_t mn = cur;
#pragma unroll
    for (int o = 8; o; o >>= 1) mn = min(mn, (uint32_t)__shfl_xor((int)mn, o, 16));
    if (mn == 0xFFFFFFFFu) break;  // uniform within the quarter
    const bool take = cur == mn;
    exc_cnt[(size_t)(base + e) * 16 + r] = take ? v.hi_cnt[p] : (uint16_t)0;
    if (r == 0) exc_ids[base + e] = (uint16_t)mn;
    if (take) p++;
    e++;
  }
  if (active && r == 0) exc_n[gq] = e;
}

hipError_t launch_exc_build(hipStream_t st, const Segs &sg, uint32_t nblocks,
                            const uint32_t *rowpos, const uint32_t *exc_off, uint32_t *exc_n,
                            uint16_t *exc_ids, uint16_t *exc_cnt) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL(exc_build_kernel, dim3((nblocks + 3) / 4), dim3(64), 0, st, sg, nblocks,
                     rowpos, exc_off, exc_n, exc_ids, exc_cnt);
  return hipGetLastError();
}

// exc_off for arbitrary row lists (blocks of 16 entries of rowpos).
__global__ __launch_bounds__(1024) void exc_offsets_kernel(SetView v,
                                                           const uint32_t *__restrict__ rowpos,
                                                           uint32_t nrows,
                                                           uint32_t *__restrict__ exc_off) {
  __shared__ uint32_t wsum[16];
  const uint32_t nb = (nrows + 15) / 16;
  uint32_t carry = 0;
  for (uint32_t b = 0; b < nb; b += 1024) {
    const uint32_t blk = b + threadIdx.x;
    uint32_t c = 0;
    if (blk < nb) {
      for (int r = 0; r < 16; r++) {
        const uint32_t s = rowpos[16u * blk + r];
        if (s != 0xFFFFFFFFu) c += v.hi_off[s + 1] - v.hi_off[s];
      }
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024>(c, wsum, tot);
    if (blk < nb) exc_off[blk] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) exc_off[nb] = carry;
}

hipError_t launch_exc_offsets(hipStream_t st, const SetView &v, const uint32_t *rowpos,
                              uint32_t nrows, uint32_t *exc_off) {
  hipLaunchKernelGGL(exc_offsets_kernel, dim3(1), dim3(1024), 0, st, v, rowpos, nrows, exc_off);
  return hipGetLastError();
}

// pos[16 * ceil(n/16)]: sorted positions of input indices first..first+n-1,
// padded with 0xFFFFFFFF.
__global__ void map_positions_kernel(const uint32_t *__restrict__ inv, uint32_t first, uint32_t n,
                                     uint32_t *__restrict__ pos) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t tot = (n + 15) / 16 * 16;
  if (t < tot) pos[t] = t < n ? inv[first + t] : 0xFFFFFFFFu;
}

hipError_t launch_map_positions(hipStream_t st, const uint32_t *inv, uint32_t first, uint32_t n,
                                uint32_t *pos) {
  const uint32_t tot = (n + 15) / 16 * 16;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(map_positions_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, inv, first,
                     n, pos);
  return hipGetLastError();
}

__global__ void fill_u64_kernel(unsigned long long *p, uint64_t n, unsigned long long value) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (uint64_t)gridDim.x * blockDim.x)
    p[t] = value;
}

hipError_t launch_fill_u64(hipStream_t st, void *p, uint64_t n_words, uint64_t value) {
  if (n_words == 0) return hipSuccess;
  uint64_t blocks = (n_words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((uint32_t)blocks), dim3(256), 0, st,
                     (unsigned long long *)p, n_words, (unsigned long long)value);
  return hipGetLastError();
}

// ---------------------------------------------------------------- export

__global__ void export_offsets_kernel(const uint32_t *__restrict__ Dorig, uint32_t N,
                                      uint64_t *__restrict__ off) {
  __shared__ unsigned long long wsum[16];
  unsigned long long carry = 0;
  for (uint32_t b = 0; b < N; b += 1024) {
    const uint32_t i = b + threadIdx.x;
    unsigned long long d = i < N ? Dorig[i] : 0;
    unsigned long long tot;
    const unsigned long long ex = block_exclusive_scan64<1024>(d, wsum, tot);
    if (i < N) off[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) off[N] = carry;
}

__global__ void export_copy_kernel(const uint64_t *__restrict__ in_off,
                                   const uint16_t *__restrict__ cap_ids,
                                   const uint16_t *__restrict__ cap_cnt,
                                   const uint32_t *__restrict__ Dorig, uint32_t N,
                                   const uint64_t *__restrict__ off, uint16_t *__restrict__ ids,
                                   uint16_t *__restrict__ counts) {
  const uint32_t i = blockIdx.x;
  if (i >= N) return;
  const uint64_t co = in_off[i] - 5ull * i;
  const uint64_t o = off[i];
  for (uint32_t t = threadIdx.x; t < Dorig[i]; t += blockDim.x) {
    ids[o + t] = cap_ids[co + t];
    counts[o + t] = cap_cnt[co + t];
  }
}

__global__ void export_dense_kernel(const uint64_t *__restrict__ in_off,
                                    const uint16_t *__restrict__ cap_ids,
                                    const uint16_t *__restrict__ cap_cnt,
                                    const uint32_t *__restrict__ Dorig, uint32_t first,
                                    uint16_t *__restrict__ out) {
  const uint32_t q = blockIdx.x, i = first + q;
  uint16_t *row = out + (size_t)q * kWords;
  for (uint32_t x = threadIdx.x; x < (uint32_t)kWords; x += blockDim.x) row[x] = 0;
  __syncthreads();
  const uint64_t co = in_off[i] - 5ull * i;
  for (uint32_t t = threadIdx.x; t < Dorig[i]; t += blockDim.x) row[cap_ids[co + t]] = cap_cnt[co + t];
}

hipError_t launch_export_lists(hipStream_t st, const kd_set *s, uint16_t *ids, uint16_t *counts,
                               uint64_t *off) {
  const uint32_t N = s->v.N;
  hipLaunchKernelGGL(export_offsets_kernel, dim3(1), dim3(1024), 0, st, s->Dorig, N, off);
  KD_HIP(hipGetLastError());
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(export_copy_kernel, dim3(N), dim3(64), 0, st, s->in_off, s->cap_ids,
                     s->cap_cnt, s->Dorig, N, off, ids, counts);
  return hipGetLastError();
}

hipError_t launch_export_dense(hipStream_t st, const kd_set *s, uint32_t first, uint32_t count,
                               uint16_t *out) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(export_dense_kernel, dim3(count), dim3(256), 0, st, s->in_off, s->cap_ids,
                     s->cap_cnt, s->Dorig, first, out);
  return hipGetLastError();
}

}  // namespace kd
