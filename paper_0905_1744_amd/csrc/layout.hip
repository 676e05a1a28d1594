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
#include <algorithm>

#include "radix.h"
#include "tilerank.h"

namespace kd {

// Sets of at most kBitonicSortMax sequences: one workgroup per set sorts
// the unique keys (key << 15) | local index (key < 2^16) with a bitonic
// network in LDS; ties in key keep index order because the index is part
// of the sort key.  (Beyond a few thousand keys the network's barrier
// count makes the radix sort below faster.)
constexpr uint32_t kBitonicSortMax = 2048;

__host__ __device__ inline uint32_t pow2_at_least(uint32_t n) {
  uint32_t p = 2;
  while (p < n) p <<= 1;
  return p;
}

// In-place ascending bitonic sort of P (a power of two) u32 values in LDS.
__device__ inline void bitonic_lds(uint32_t *sk, uint32_t P, uint32_t nt) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t x = tid; x < (P >> 1); x += nt) {
        const uint32_t a = ((x & ~(j - 1)) << 1) | (x & (j - 1));
        const uint32_t b = a | j;
        const uint32_t va = sk[a], vb = sk[b];
        if ((va > vb) == ((a & k) == 0)) {
          sk[a] = vb;
          sk[b] = va;
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(1024) void sort_small_kernel(const uint32_t *__restrict__ keys,
                                                          const uint32_t *__restrict__ seq,
                                                          uint32_t *__restrict__ perm) {
  extern __shared__ uint32_t sk[];
  const uint32_t a = seq[blockIdx.x], n = seq[blockIdx.x + 1] - a;
  if (n == 0 || n > kBitonicSortMax) return;
  const uint32_t P = pow2_at_least(n);
  for (uint32_t t = threadIdx.x; t < P; t += 1024) sk[t] = t < n ? (keys[a + t] << 15) | t : 0xFFFFFFFFu;
  __syncthreads();
  bitonic_lds(sk, P, 1024);
  for (uint32_t t = threadIdx.x; t < n; t += 1024) perm[a + t] = sk[t] & 0x7FFFu;
}

// Larger sets: each key's position in the stable order comes from ranking
// it against sorted tiles of the set's keys (tilerank.h), then a scatter.
struct SetKeyOf {
  const uint32_t *keys;
  __device__ unsigned long long operator()(uint32_t i) const { return keys[i]; }
};

__global__ __launch_bounds__(256) void scatter_perm_kernel(uint32_t n, const uint32_t *__restrict__ rank,
                                                           uint32_t *__restrict__ perm) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) perm[rank[i]] = i;
}

hipError_t launch_sort_u32_index(hipStream_t st, const uint32_t *keys, const Segs &sg,
                                 const uint32_t *host_first, uint32_t *perm, void *scratch) {
  uint32_t max_n = 0;
  for (uint32_t q = 0; q < sg.nsets; q++) max_n = std::max(max_n, host_first[q + 1] - host_first[q]);
  if (max_n == 0) return hipSuccess;
  const uint32_t small_max = max_n < kBitonicSortMax ? max_n : kBitonicSortMax;
  hipLaunchKernelGGL(sort_small_kernel, dim3(sg.nsets), dim3(1024),
                     sizeof(uint32_t) * pow2_at_least(small_max), st, keys, sg.seq, perm);
  KD_HIP(hipGetLastError());
  if (max_n <= kBitonicSortMax) return hipSuccess;
  KeyIdx *sorted = static_cast<KeyIdx *>(scratch);
  uint32_t *rank = reinterpret_cast<uint32_t *>(sorted + max_n);
  for (uint32_t q = 0; q < sg.nsets; q++) {
    const uint32_t a = host_first[q], n = host_first[q + 1] - a;
    if (n <= kBitonicSortMax) continue;
    KD_HIP(launch_tile_rank(st, SetKeyOf{keys + a}, n, sorted, rank));
    hipLaunchKernelGGL(scatter_perm_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, rank, perm + a);
    KD_HIP(hipGetLastError());
  }
  return hipSuccess;
}

size_t sort_scratch_bytes(uint32_t max_n) { return (sizeof(KeyIdx) + 4) * (size_t)max_n + 256; }

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
  const uint32_t a = sg.seq[sg.set_of_pos(s)];
  const uint32_t i = a + perm[s];
  inv[i] = s - a;
  K[s] = Korig[i];
  invK[s] = 1.0 / (double)Korig[i];
  D[s] = Dorig[i];
  hcount[s] = nhi_orig[i];
}

// Per batch-wide column group (one wave each): padded list length (the
// group's longest list, i.e. its last: D ascending, rounded to 16), longest
// count>=2 list (rounded to 4), and the count>=2 entries of each of its
// four row blocks.  Each workgroup also leaves the sum of D and the longest
// padded list of its four groups in part_ent / part_max.
__global__ __launch_bounds__(256) void layout_groups_meta_kernel(
    Segs sg, uint32_t G, const uint32_t *__restrict__ D, const uint32_t *__restrict__ hcount,
    uint32_t *__restrict__ grp_len, uint32_t *__restrict__ ghi_len, uint32_t *__restrict__ rbcnt,
    const unsigned long long *err, unsigned long long *part_ent, unsigned long long *part_max) {
  __shared__ unsigned long long s_ent[4], s_max[4];
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t x = blockIdx.x * 4 + w, lane = threadIdx.x & 63u;
  if (*err != ~0ull) return;  // the same for every workgroup
  unsigned long long sd = 0, L = 0;
  if (x < G) {
    const uint32_t s = sg.set_of_grp(x);
    const uint32_t a = sg.seq[s], n = sg.seq[s + 1] - a, g = x - sg.grp[s];
    const bool valid = 64u * g + lane < n;
    const uint32_t h = valid ? hcount[a + 64u * g + lane] : 0u;
    const uint32_t d = valid ? D[a + 64u * g + lane] : 0u;
    uint32_t mh = h, md = d, rs = h;
    sd = d;
#pragma unroll
    for (int o = 32; o; o >>= 1) {
      mh = max(mh, (uint32_t)__shfl_xor((int)mh, o, 64));
      md = max(md, (uint32_t)__shfl_xor((int)md, o, 64));
      sd += __shfl_xor(sd, o, 64);
    }
#pragma unroll
    for (int o = 8; o; o >>= 1) rs += (uint32_t)__shfl_xor((int)rs, o, 16);
    L = (md + 15u) & ~15u;
    if (lane == 0) {
      grp_len[x] = (uint32_t)L;
      ghi_len[x] = (mh + 3u) & ~3u;
    }
    const uint32_t rb = 4u * g + (lane >> 4);
    if ((lane & 15u) == 0 && 16u * rb < n) rbcnt[sg.rb[s] + rb] = rs;
  }
  if (lane == 0) {
    s_ent[w] = sd;
    s_max[w] = L;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part_ent[blockIdx.x] = s_ent[0] + s_ent[1] + s_ent[2] + s_ent[3];
    part_max[blockIdx.x] = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
  }
}

// Exclusive scans of four arrays at once (y = which): hi_off over the
// sorted positions, grp_off and ghi_off (64 x length) over the column
// groups, exc_off over the row blocks.  Three passes: tile sums, a scan of
// the tile sums (which also writes the totals), the scan of each tile.
constexpr uint32_t kScanTile = 4096;  // 1024 threads x 4 values

struct ScanJob {
  const uint32_t *in;
  uint32_t n;
  uint32_t mul;
  uint32_t *out32;  // one of out32 / out64
  uint64_t *out64;
};
struct ScanJobs {
  ScanJob j[4];
  unsigned long long *part;  // [4][nblk] tile sums, then tile offsets
  uint32_t nblk;
  uint32_t npart;            // per-workgroup group statistics
  const unsigned long long *part_ent, *part_max;
};

__global__ __launch_bounds__(1024) void scan_tiles_kernel(ScanJobs J, const unsigned long long *err) {
  __shared__ unsigned long long wsum[16];
  const ScanJob jb = J.j[blockIdx.y];
  const uint32_t x0 = blockIdx.x * kScanTile;
  if (x0 >= jb.n || *err != ~0ull) return;
  unsigned long long v = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t x = x0 + 4u * threadIdx.x + k;
    if (x < jb.n) v += (unsigned long long)jb.in[x] * jb.mul;
  }
  unsigned long long tot;
  block_exclusive_scan64<1024>(v, wsum, tot);
  if (threadIdx.x == 0) J.part[blockIdx.y * J.nblk + blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void scan_top_kernel(ScanJobs J, const unsigned long long *err,
                                                        LayoutMeta *meta) {
  __shared__ unsigned long long wsum[16];
  const uint32_t y = blockIdx.x;
  if (*err != ~0ull) {
    if (y == 0 && threadIdx.x == 0) meta->err = *err;
    return;
  }
  if (y == 0) {  // totals of the per-workgroup group statistics
    unsigned long long e = 0, m = 0;
    for (uint32_t b = threadIdx.x; b < J.npart; b += 1024) {
      e += J.part_ent[b];
      m = max(m, J.part_max[b]);
    }
#pragma unroll
    for (int o = 32; o; o >>= 1) {
      e += __shfl_xor(e, o, 64);
      m = max(m, (unsigned long long)__shfl_xor(m, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&meta->entries, e);
      atomicMax(&meta->max_len, m);
    }
  }
  const ScanJob jb = J.j[y];
  const uint32_t nb = (jb.n + kScanTile - 1) / kScanTile;
  unsigned long long *part = J.part + y * J.nblk;
  unsigned long long carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
    const uint32_t b = b0 + threadIdx.x;
    const unsigned long long v = b < nb ? part[b] : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block_exclusive_scan64<1024>(v, wsum, tot);
    if (b < nb) part[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (jb.out32) jb.out32[jb.n] = (uint32_t)carry;
    else jb.out64[jb.n] = carry;
    if (y == 0) meta->n_hi = carry;
    if (y == 1) meta->n_gids = carry;
    if (y == 2) meta->n_ghi = carry;
    if (y == 3) meta->n_exc = carry;
    if (y == 0) meta->err = ~0ull;
  }
}

__global__ __launch_bounds__(1024) void scan_write_kernel(ScanJobs J, const unsigned long long *err) {
  __shared__ unsigned long long wsum[16];
  const ScanJob jb = J.j[blockIdx.y];
  const uint32_t x0 = blockIdx.x * kScanTile;
  if (x0 >= jb.n || *err != ~0ull) return;
  unsigned long long v[4], loc = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t x = x0 + 4u * threadIdx.x + k;
    v[k] = x < jb.n ? (unsigned long long)jb.in[x] * jb.mul : 0ull;
    loc += v[k];
  }
  unsigned long long tot;
  unsigned long long run = J.part[blockIdx.y * J.nblk + blockIdx.x] + block_exclusive_scan64<1024>(loc, wsum, tot);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const uint32_t x = x0 + 4u * threadIdx.x + k;
    if (x < jb.n) {
      if (jb.out32) jb.out32[x] = (uint32_t)run;
      else jb.out64[x] = run;
    }
    run += v[k];
  }
}

size_t layout_meta_scratch_bytes(uint32_t N, uint32_t G, uint32_t RB) {
  const uint32_t nblk = (N + kScanTile - 1) / kScanTile;
  const uint64_t npart = (G + 3) / 4;
  return 4ull * RB + 256 + 8ull * 4 * (nblk ? nblk : 1) + 16ull * npart + 256;
}

hipError_t launch_layout_meta(hipStream_t st, const Segs &sg, uint32_t N, uint32_t G,
                              uint32_t RB, const uint32_t *perm,
                              const uint32_t *Dorig, const uint32_t *Korig,
                              const uint32_t *nhi_orig, uint32_t *inv, uint32_t *K, uint32_t *D,
                              double *invK, uint32_t *hcount, uint32_t *hi_off, uint64_t *grp_off,
                              uint32_t *grp_len, uint64_t *ghi_off, uint32_t *ghi_len,
                              uint32_t *exc_off, const unsigned long long *err, LayoutMeta *meta,
                              void *scratch) {
  uint32_t *rbcnt = static_cast<uint32_t *>(scratch);
  const uint32_t nblk = (N + kScanTile - 1) / kScanTile;  // N >= G, RB
  ScanJobs J;
  J.part = reinterpret_cast<unsigned long long *>(static_cast<char *>(scratch) +
                                                  ((4ull * RB + 255) & ~255ull));
  J.nblk = nblk;
  J.j[0] = {hcount, N, 1u, hi_off, nullptr};
  J.j[1] = {grp_len, G, 64u, nullptr, grp_off};
  J.j[2] = {ghi_len, G, 64u, nullptr, ghi_off};
  J.j[3] = {rbcnt, RB, 1u, exc_off, nullptr};
  const uint32_t npart = (G + 3) / 4;
  unsigned long long *pe = J.part + 4ull * (nblk ? nblk : 1);
  J.npart = npart;
  J.part_ent = pe;
  J.part_max = pe + npart;
  hipLaunchKernelGGL(layout_gather_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sg, N, perm,
                     Dorig, Korig, nhi_orig, inv, K, D, invK, hcount, err);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(layout_groups_meta_kernel, dim3(npart), dim3(256), 0, st, sg, G, D,
                     hcount, grp_len, ghi_len, rbcnt, err, pe, pe + npart);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(nblk, 4), dim3(1024), 0, st, J, err);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_top_kernel, dim3(4), dim3(1024), 0, st, J, err, meta);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(scan_write_kernel, dim3(nblk, 4), dim3(1024), 0, st, J, err);
  return hipGetLastError();
}

// Grid (batch-wide column group, slice y of kGroupSlices), 256 threads.
// The group's 64 lists are copied in slices of 128 words through LDS: a
// wave reads 64 consecutive words of one list per load (coalesced), then
// lane l writes its list's 16-byte chunks into the interleaved layout (the
// 64 lanes' chunks adjacent: coalesced 1 KB stores).  Words past a list's
// end are the sentinel.  Workgroup y takes slices y, y + kGroupSlices, ...
constexpr uint32_t kGroupSlices = 4;
constexpr uint32_t kSliceWords = 128;

__global__ __launch_bounds__(256) void layout_groups_kernel(Segs sg,
                                                            const uint64_t *__restrict__ offsets,
                                                            const uint16_t *__restrict__ cap_ids,
                                                            uint16_t *__restrict__ gids) {
  typedef __attribute__((address_space(1))) const uint16_t gcu16;  // global loads, not flat
  __shared__ uint16_t buf[64][kSliceWords + 8];  // padded rows: 16-byte reads stay aligned
  __shared__ const uint16_t *src[64];
  __shared__ uint32_t len[64];
  const uint32_t x = blockIdx.x, tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t set = sg.set_of_grp(x);
  const SetView &v = sg.views[set];
  const uint32_t g = x - sg.grp[set];
  const uint32_t L = v.grp_len[g];
  if (blockIdx.y * kSliceWords >= L) return;  // uniform: nothing for this workgroup
  if (tid < 64) {
    const uint32_t s = 64u * g + tid;
    src[tid] = cap_ids;  // an empty list: any valid address, never used
    len[tid] = 0;
    if (s < v.N) {
      const uint32_t i = v.base + v.perm[s];
      src[tid] = cap_ids + (offsets[i] - 5ull * i);
      len[tid] = v.D[s];
    }
  }
  __syncthreads();
  uint4 *dst = reinterpret_cast<uint4 *>(gids + v.grp_off[g]);
  for (uint32_t t0 = blockIdx.y * kSliceWords; t0 < L; t0 += kGroupSlices * kSliceWords) {
    // wave w loads lists w, w + 4, ..., w + 60: 64 words per instruction,
    // two per list, all 32 loads issued before the first LDS write (indices
    // clamped into the list, so no load is conditional)
    constexpr uint32_t kHalves = kSliceWords / 64;
    uint32_t val[16][kHalves], n[16];
#pragma unroll
    for (uint32_t k = 0; k < 16; k++) {
      const uint32_t r = wave + 4u * k;
      gcu16 *sp = (gcu16 *)src[r];
      n[k] = len[r];
#pragma unroll
      for (uint32_t h = 0; h < kHalves; h++) {
        const uint32_t t = t0 + 64u * h + lane;
        val[k][h] = sp[t < n[k] ? t : 0u];
      }
    }
#pragma unroll
    for (uint32_t k = 0; k < 16; k++) {
#pragma unroll
      for (uint32_t h = 0; h < kHalves; h++) {
        const uint32_t t = t0 + 64u * h + lane;
        buf[wave + 4u * k][64u * h + lane] = t < n[k] ? (uint16_t)val[k][h] : (uint16_t)kSentinel;
      }
    }
    __syncthreads();
    // lane l = list l; wave w writes chunks w, w + 4, ... of the slice
    const uint32_t nch = min(kSliceWords, L - t0) / 8;  // L is a multiple of 16
    for (uint32_t c = wave; c < nch; c += 4) {
      const uint4 q = *reinterpret_cast<const uint4 *>(&buf[lane][8 * c]);
      dst[(size_t)(t0 / 8 + c) * 64 + lane] = q;
    }
    __syncthreads();
  }
}

// One thread per batch-wide sorted position: its count>=2 entries (packed,
// from the counting pass) into the CSR lists and the group-interleaved list.
__global__ __launch_bounds__(256) void layout_hi_kernel(Segs sg, uint32_t N,
                                                        const uint64_t *__restrict__ offsets,
                                                        const uint32_t *__restrict__ hi_cap,
                                                        uint16_t *__restrict__ hi_ids,
                                                        uint16_t *__restrict__ hi_cnt,
                                                        uint32_t *__restrict__ ghi) {
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= N) return;
  const uint32_t set = sg.set_of_pos(p);
  const SetView &v = sg.views[set];
  const uint32_t s = p - v.base;
  const uint32_t h0 = v.hi_off[s], nh = v.hi_off[s + 1] - h0;
  if (nh == 0) return;
  const uint32_t i = v.base + v.perm[s];
  const uint32_t *src = hi_cap + (offsets[i] - 5ull * i);
  uint32_t *gdst = ghi + v.ghi_off[s >> 6] + (s & 63u);
  for (uint32_t t = 0; t < nh; t++) {
    const uint32_t e = src[t];
    hi_ids[h0 + t] = (uint16_t)e;
    hi_cnt[h0 + t] = (uint16_t)(e >> 16);
    gdst[64ull * t] = e;
  }
}

hipError_t launch_layout_fill(hipStream_t st, const Segs &sg, const SetView &v,
                              const uint64_t *offsets,
                              const uint16_t *cap_ids, const uint32_t *hi_cap, uint16_t *gids,
                              uint16_t *hi_ids, uint16_t *hi_cnt, uint32_t *ghi,
                              uint32_t max_len) {
  (void)max_len;
  if (v.N == 0) return hipSuccess;
  hipLaunchKernelGGL(layout_groups_kernel, dim3(v.G, kGroupSlices), dim3(256), 0, st, sg, offsets,
                     cap_ids, gids);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(layout_hi_kernel, dim3((v.N + 255) / 256), dim3(256), 0, st, sg, v.N, offsets,
                     hi_cap, hi_ids, hi_cnt, ghi);
  return hipGetLastError();
}

// Merged count>=2 words of a row block by a quarter-wave (16 lanes, one
// per row): each lane walks its row's sorted list (sorted position s, or
// 0xFFFFFFFF for none), the quarter agrees on the smallest pending word,
// and every lane writes its row's count for it (0 when the row lacks it).
// Returns the number of merged words.
__device__ inline uint32_t merge_rows(const SetView &v, uint32_t s, uint32_t r, uint32_t base,
                                      uint16_t *__restrict__ exc_ids,
                                      uint16_t *__restrict__ exc_cnt) {
  uint32_t p = 0, pe = 0;
  if (s != 0xFFFFFFFFu) {
    p = v.hi_off[s];
    pe = v.hi_off[s + 1];
  }
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
  return e;
}

// Listed rows (block b = sorted positions rowpos[16b .. 16b+15] of the first
// set): one quarter-wave per block.
__global__ __launch_bounds__(64) void exc_build_kernel(Segs sg, uint32_t nblocks,
                                                        const uint32_t *__restrict__ rowpos,
                                                        const uint32_t *__restrict__ exc_off,
                                                        uint32_t *__restrict__ exc_n,
                                                        uint16_t *__restrict__ exc_ids,
                                                        uint16_t *__restrict__ exc_cnt) {
  const uint32_t gq = blockIdx.x * 4 + (threadIdx.x >> 4);  // block handled by this quarter
  const uint32_t r = threadIdx.x & 15;
  const bool active = gq < nblocks;
  const uint32_t s = active ? rowpos[16u * gq + r] : 0xFFFFFFFFu;
  const uint32_t e = merge_rows(sg.views[0], s, r, active ? exc_off[gq] : 0u, exc_ids, exc_cnt);
  if (active && r == 0) exc_n[gq] = e;
}

// Every row block of every set (batch-wide numbering), one wave each.  The
// 16 rows are consecutive sorted positions, so their count>=2 entries are
// one contiguous range; up to kExcStage of them are staged in LDS as keys
// (word, row, slot), sorted, and each distinct word emits its 16 counts.
// Larger blocks (rare) fall back to the quarter-wave merge.
constexpr uint32_t kExcStage = 512;

__global__ __launch_bounds__(64) void exc_build_rows_kernel(Segs sg,
                                                            const uint32_t *__restrict__ exc_off,
                                                            uint32_t *__restrict__ exc_n,
                                                            uint16_t *__restrict__ exc_ids,
                                                            uint16_t *__restrict__ exc_cnt) {
  __shared__ uint32_t key[kExcStage];
  __shared__ uint16_t cv[kExcStage];
  __shared__ uint16_t ust[kExcStage];
  __shared__ uint32_t roff[17];
  const uint32_t gq = blockIdx.x, lane = threadIdx.x;
  const uint32_t set = sg.set_of_rb(gq);
  const SetView &v = sg.views[set];
  const uint32_t n = sg.seq[set + 1] - sg.seq[set];
  const uint32_t s0 = 16u * (gq - sg.rb[set]), s1 = min(s0 + 16u, n);
  if (lane <= 16u) roff[lane] = v.hi_off[min(s0 + lane, s1)];
  __syncthreads();
  const uint32_t e0 = roff[0], T = roff[16] - e0;
  const uint32_t base = exc_off[gq];
  if (T > kExcStage) {
    if (lane < 16u) {
      const uint32_t e = merge_rows(v, s0 + lane < s1 ? s0 + lane : 0xFFFFFFFFu, lane, base,
                                    exc_ids, exc_cnt);
      if (lane == 0) exc_n[gq] = e;
    }
    return;
  }
  if (T == 0) {
    if (lane == 0) exc_n[gq] = 0;
    return;
  }
  const uint32_t P = pow2_at_least(T);
  for (uint32_t t = lane; t < P; t += 64) {
    uint32_t k = 0xFFFFFFFFu;
    if (t < T) {
      const uint32_t x = e0 + t;
      uint32_t r = 0;
#pragma unroll
      for (int q = 1; q < 16; q++) r += roff[q] <= x;
      k = ((uint32_t)v.hi_ids[x] << 13) | (r << 9) | t;
      cv[t] = v.hi_cnt[x];
    }
    key[t] = k;
  }
  __syncthreads();
  bitonic_lds(key, P, 64);
  // distinct words: each lane takes a contiguous run of sorted slots
  const uint32_t per = (T + 63) / 64, t0 = min(lane * per, T), t1 = min(t0 + per, T);
  uint32_t nf = 0;
  for (uint32_t t = t0; t < t1; t++) nf += (t == 0 || (key[t] >> 13) != (key[t - 1] >> 13));
  uint32_t incl = nf;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += y;
  }
  const uint32_t nu = __shfl(incl, 63, 64);
  uint32_t u = incl - nf;
  for (uint32_t t = t0; t < t1; t++)
    if (t == 0 || (key[t] >> 13) != (key[t - 1] >> 13)) ust[u++] = (uint16_t)t;
  __syncthreads();
  for (uint32_t w = lane; w < nu; w += 64) {
    uint32_t t = ust[w];
    const uint32_t id = key[t] >> 13;
    uint16_t *row = exc_cnt + (size_t)(base + w) * 16;
    uint4 *row4 = reinterpret_cast<uint4 *>(row);
    row4[0] = make_uint4(0u, 0u, 0u, 0u);
    row4[1] = make_uint4(0u, 0u, 0u, 0u);
    for (; t < T && (key[t] >> 13) == id; t++) row[(key[t] >> 9) & 15u] = cv[key[t] & 511u];
    exc_ids[base + w] = (uint16_t)id;
  }
  if (lane == 0) exc_n[gq] = nu;
}

hipError_t launch_exc_build(hipStream_t st, const Segs &sg, uint32_t nblocks,
                            const uint32_t *rowpos, const uint32_t *exc_off, uint32_t *exc_n,
                            uint16_t *exc_ids, uint16_t *exc_cnt) {
  if (nblocks == 0) return hipSuccess;
  if (rowpos)
    hipLaunchKernelGGL(exc_build_kernel, dim3((nblocks + 3) / 4), dim3(64), 0, st, sg, nblocks,
                       rowpos, exc_off, exc_n, exc_ids, exc_cnt);
  else
    hipLaunchKernelGGL(exc_build_rows_kernel, dim3(nblocks), dim3(64), 0, st, sg, exc_off, exc_n,
                       exc_ids, exc_cnt);
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

// Globalized rank, Algorithm 2 step 4: the k samples of each set are the
// sequences at 0-based positions floor(t w / (k+1)), t = 1..k, of the set's
// w sequences in key order.
__global__ void pick_samples_kernel(const uint32_t *__restrict__ first, uint32_t nsets, uint32_t k,
                                    const uint32_t *__restrict__ order, uint32_t *__restrict__ samples) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nsets * k) return;
  const uint32_t q = x / k, t = x % k + 1u;
  const uint32_t a = first[q], w = first[q + 1] - a;
  samples[x] = a + order[a + (uint32_t)((uint64_t)t * w / (k + 1u))];
}

hipError_t launch_pick_samples(hipStream_t st, const uint32_t *first, uint32_t nsets, uint32_t k,
                               const uint32_t *order, uint32_t *samples) {
  const uint32_t n = nsets * k;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(pick_samples_kernel, dim3((n + 255) / 256), dim3(256), 0, st, first, nsets, k,
                     order, samples);
  return hipGetLastError();
}

// Step 5: the sample set's per-input arrays, one wave per sample.  Its
// distinct-word lists are the parent's (same capacity base), its count>=2
// entries are re-packed from the parent's sorted-order lists.
__global__ __launch_bounds__(256) void gather_samples_kernel(
    Segs par, const uint64_t *__restrict__ par_in_off, const uint32_t *__restrict__ par_Dorig,
    const uint32_t *__restrict__ picks, uint32_t S, uint64_t *__restrict__ in_off,
    uint32_t *__restrict__ Dorig, uint32_t *__restrict__ Korig, uint32_t *__restrict__ nhi,
    uint32_t *__restrict__ hi_cap) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t s = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (s >= S) return;
  const uint32_t i = picks[s];
  const uint32_t q = par.set_of_pos(i), a = par.seq[q];
  const SetView &v = par.views[q];
  const uint32_t p = v.inv[i - a];
  const uint32_t h0 = v.hi_off[p], nh = v.hi_off[p + 1] - h0;
  const uint64_t co = par_in_off[i] - 5ull * i;
  for (uint32_t t = lane; t < nh; t += 64)
    hi_cap[co + t] = (uint32_t)v.hi_ids[h0 + t] | ((uint32_t)v.hi_cnt[h0 + t] << 16);
  if (lane == 0) {
    in_off[s] = co + 5ull * s;
    Dorig[s] = par_Dorig[i];
    Korig[s] = (uint32_t)(par_in_off[i + 1] - par_in_off[i]) - 5u;
    nhi[s] = nh;
  }
}

hipError_t launch_gather_samples(hipStream_t st, const Segs &parent, const uint64_t *par_in_off,
                                 const uint32_t *par_Dorig, const uint32_t *picks, uint32_t S,
                                 uint64_t *in_off, uint32_t *Dorig, uint32_t *Korig,
                                 uint32_t *nhi, uint32_t *hi_cap) {
  if (S == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_samples_kernel, dim3((S + 3) / 4), dim3(256), 0, st, parent, par_in_off,
                     par_Dorig, picks, S, in_off, Dorig, Korig, nhi, hi_cap);
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

// one workgroup per set writes its id over its positions, groups and row blocks
__global__ __launch_bounds__(256) void seg_ids_kernel(Segs sg, uint32_t *__restrict__ pos_set,
                                                      uint32_t *__restrict__ grp_set,
                                                      uint32_t *__restrict__ rb_set) {
  const uint32_t s = blockIdx.x;
  for (uint32_t p = sg.seq[s] + threadIdx.x; p < sg.seq[s + 1]; p += 256) pos_set[p] = s;
  for (uint32_t x = sg.grp[s] + threadIdx.x; x < sg.grp[s + 1]; x += 256) grp_set[x] = s;
  for (uint32_t x = sg.rb[s] + threadIdx.x; x < sg.rb[s + 1]; x += 256) rb_set[x] = s;
}

hipError_t launch_seg_ids(hipStream_t st, const Segs &sg, uint32_t *pos_set, uint32_t *grp_set,
                          uint32_t *rb_set) {
  hipLaunchKernelGGL(seg_ids_kernel, dim3(sg.nsets), dim3(256), 0, st, sg, pos_set, grp_set, rb_set);
  return hipGetLastError();
}

__global__ void fill_multi_kernel(FillJobs J) {
  const FillJob f = J.j[blockIdx.y];
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < f.n;
       t += (uint64_t)gridDim.x * blockDim.x)
    f.p[t] = f.v;
}

hipError_t launch_fills(hipStream_t st, const FillJobs &J) {
  uint64_t mx = 0;
  for (uint32_t q = 0; q < J.n; q++) mx = std::max<uint64_t>(mx, J.j[q].n);
  if (mx == 0) return hipSuccess;
  uint64_t blocks = (mx + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_multi_kernel, dim3((uint32_t)blocks, J.n), dim3(256), 0, st, J);
  return hipGetLastError();
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
