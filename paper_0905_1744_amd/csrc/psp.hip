// Profiles and the profile sum of pairs score (paper Section 3.1.3,
// Equation 4): PSP(x, y) = sum_i sum_j fX[x][i] fY[y][j] M[i][j] for every
// column x of profile X and column y of profile Y, M[i][j] = log(p_ij /
// (p_i p_j)) supplied by the caller.  As matrices, S = fX M fY^T: a dense
// contraction with K = 20, done on the matrix cores in FP64
// (v_mfma_f64_16x16x4_f64, five K-steps of 4).
#include <vector>

#include "kd_internal.h"

namespace kd {

// --------------------------------------------------------------- profiles

// one thread per column; counts in LDS ([amino acid][thread], no bank
// conflicts); f = count / m.  A byte that is neither an amino acid nor a
// gap records its row-major position in *bad (smallest wins).
__global__ __launch_bounds__(256) void psp_profile_kernel(const uint8_t *__restrict__ aln, uint32_t m,
                                                          uint32_t L, double *__restrict__ f,
                                                          unsigned long long *bad) {
  __shared__ uint32_t cnt[20][256];
  __shared__ int8_t code[256];
  const uint32_t t = threadIdx.x;
  {
    // 20 amino acids in the order of their one-letter codes; gaps -2
    const char *order = "ACDEFGHIKLMNPQRSTVWY";
    int8_t c = -1;
    for (int a = 0; a < 20; a++)
      if ((uint32_t)(uint8_t)order[a] == t) c = (int8_t)a;
    if (t == '-' || t == '.') c = -2;
    code[t] = c;
  }
  for (int a = 0; a < 20; a++) cnt[a][t] = 0;
  __syncthreads();
  const uint32_t x = blockIdx.x * 256u + t;
  if (x >= L) return;
  for (uint32_t r = 0; r < m; r++) {
    const uint64_t pos = (uint64_t)r * L + x;
    const int c = code[aln[pos]];
    if (c >= 0) cnt[c][t]++;
    else if (c == -1) {
      atomicMin(bad, (unsigned long long)pos);
      break;
    }
  }
  for (int a = 0; a < 20; a++) f[(uint64_t)x * 20 + a] = (double)cnt[a][t] / (double)m;
}

hipError_t launch_psp_profile(hipStream_t st, const uint8_t *aln, uint32_t m, uint32_t L, double *f,
                              unsigned long long *bad) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(psp_profile_kernel, dim3((L + 255) / 256), dim3(256), 0, st, aln, m, L, f, bad);
  return hipGetLastError();
}

// ------------------------------------------------------------------ scores

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr uint32_t kPspRowsPerTile = 64;  // rows per score workgroup (4 waves)
constexpr uint32_t kPspRows = 16;         // rows per wave (one MFMA block high)
constexpr uint32_t kPspCols = 512;        // columns per wave

bool psp_plan(std::vector<PspWork> &w, uint64_t &gblks, uint64_t &tiles) {
  gblks = tiles = 0;
  for (auto &p : w) {
    const uint64_t rt = (p.lx + kPspRowsPerTile - 1) / kPspRowsPerTile;
    const uint64_t ct = (p.ly + kPspCols - 1) / kPspCols;
    p.gblk0 = (uint32_t)gblks;
    p.tile0 = (uint32_t)tiles;
    gblks += rt;
    tiles += rt * ct;
    if (tiles > 0x7FFFFFFFull) return false;  // beyond one launch's grid
  }
  return true;
}

// the pair whose range [first, next first) holds global block id b
template <class FirstOf>
__device__ __forceinline__ uint32_t pair_of(uint32_t npairs, uint32_t b, FirstOf first) {
  uint32_t lo = 0, hi = npairs;  // last pair with first(q) <= b
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (first(mid) <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// G = fX M for every row of every pair (the first factor of the
// contraction): a workgroup takes 64 rows of one pair (compact grid over
// all pairs' row blocks), stages their frequencies in LDS with coalesced
// loads and writes the 64 x 20 block of G contiguously; each G[x][j] is
// summed over i in fixed order.
__global__ __launch_bounds__(256) void psp_g_kernel(const PspWork *__restrict__ w, uint32_t npairs,
                                                    const double *__restrict__ M) {
  __shared__ double sM[400];
  __shared__ double sF[64 * 20];
  const uint32_t q = pair_of(npairs, blockIdx.x, [&](uint32_t i) { return w[i].gblk0; });
  const PspWork pr = w[q];
  const uint32_t r0 = (blockIdx.x - pr.gblk0) * 64u;
  const uint32_t n = min(64u, pr.lx - r0) * 20u;
  for (uint32_t e = threadIdx.x; e < 400; e += 256) sM[e] = M[e];
  for (uint32_t e = threadIdx.x; e < n; e += 256) sF[e] = pr.fx[(uint64_t)r0 * 20 + e];
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < n; e += 256) {
    const uint32_t x = e / 20u, j = e % 20u;
    double g = 0.0;
#pragma unroll
    for (int i = 0; i < 20; i++) g = fma(sF[x * 20 + i], sM[i * 20 + j], g);
    pr.g[(uint64_t)r0 * 20 + e] = g;
  }
}

// One workgroup = one tile of one pair (compact grid over all pairs'
// tiles): 64 rows x up to 512 columns, wave w taking rows 16w .. 16w+15,
// 64 columns (four 16 x 16 blocks) at a time on the matrix cores: lane l
// supplies A[l%16][l/16] = G[row][4k + l/16] and B[l/16][l%16] =
// fY[col][4k + l/16] (read straight from memory; the 64 x 20 slice of fY is
// 10 KB and stays in cache) and holds D[l/16 + 4r][l%16], r = 0..3, of each
// block.  The 16 x 64 results pass through the wave's LDS tile so that each
// store writes one row's 64 consecutive scores (512 bytes).
__global__ __launch_bounds__(256) void psp_scores_kernel(const PspWork *__restrict__ w, uint32_t npairs) {
  __shared__ double tile[4][16][65];  // per wave; +1 column against bank conflicts
  const uint32_t q = pair_of(npairs, blockIdx.x, [&](uint32_t i) { return w[i].tile0; });
  const PspWork pr = w[q];
  const uint32_t nty = (pr.ly + kPspCols - 1) / kPspCols;
  const uint32_t t = blockIdx.x - pr.tile0;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t x0 = (t / nty) * kPspRowsPerTile + wave * kPspRows, yb = (t % nty) * kPspCols;
  if (x0 >= pr.lx) return;  // the last row tile of a pair may have fewer than 64 rows
  const uint32_t li = lane & 15u, lk = lane >> 4;
  double a[5];
  {
    const uint32_t x = min(x0 + li, pr.lx - 1u);  // rows past the end: any valid row, not stored
#pragma unroll
    for (int k = 0; k < 5; k++) a[k] = pr.g[(uint64_t)x * 20 + 4 * k + lk];
  }
  const uint32_t ye = min(pr.ly, yb + kPspCols);
  for (uint32_t y0 = yb; y0 < ye; y0 += 64) {
    double b[4][5];
#pragma unroll
    for (int cb = 0; cb < 4; cb++) {
      const uint32_t y = min(y0 + 16u * cb + li, pr.ly - 1u);
#pragma unroll
      for (int k = 0; k < 5; k++) b[cb][k] = pr.fy[(uint64_t)y * 20 + 4 * k + lk];
    }
    v4d acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; cb++) {
      acc[cb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 5; k++) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k], b[cb][k], acc[cb], 0, 0, 0);
    }
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
      for (int r = 0; r < 4; r++) tile[wave][lk + 4 * r][16 * cb + li] = acc[cb][r];
    // the wave's own tile: order its writes before its reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t y = y0 + lane;
#pragma unroll
    for (int row = 0; row < 16; row++) {
      const uint32_t x = x0 + row;
      if (x < pr.lx && y < pr.ly) pr.scores[(uint64_t)x * pr.ly + y] = tile[wave][row][lane];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // reads done before the next writes
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

hipError_t launch_psp_scores(hipStream_t st, const PspWork *w, uint32_t npairs, uint32_t gblks,
                             uint32_t tiles, const double *M) {
  if (npairs == 0 || tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(psp_g_kernel, dim3(gblks), dim3(256), 0, st, w, npairs, M);
  KD_HIP(hipGetLastError());
  hipLaunchKernelGGL(psp_scores_kernel, dim3(tiles), dim3(256), 0, st, w, npairs);
  return hipGetLastError();
}

}  // namespace kd
