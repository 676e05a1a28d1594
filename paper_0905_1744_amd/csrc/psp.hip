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
// the work list's pointers name global memory: loads and stores through
// them are global (not flat) instructions, whose completion counts in order
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) double gdouble;

constexpr uint32_t kPspRowsPerTile = 64;  // rows per score workgroup; each wave takes all of them, 16 at a time
constexpr uint32_t kPspRows = 16;         // rows per step (one MFMA block high)
constexpr uint32_t kPspPieces = 4;        // 64-column pieces per workgroup, one per wave
constexpr uint32_t kPspSpan = 80;         // columns a wave computes: its piece's 64 and the 16 before

// 64-column pieces of a row of ly scores: the row is cut on 128-byte lines
// 16 columns before each multiple of 64 (see psp_scores_kernel)
__host__ __device__ inline uint32_t psp_pieces(uint32_t ly) { return (ly + 16 + 63) / 64; }

bool psp_plan(std::vector<PspWork> &w, uint64_t &gblks, uint64_t &tiles) {
  gblks = tiles = 0;
  for (auto &p : w) {
    const uint64_t rt = (p.lx + kPspRowsPerTile - 1) / kPspRowsPerTile;
    const uint64_t ct = (psp_pieces(p.ly) + kPspPieces - 1) / kPspPieces;
    p.gblk0 = (uint32_t)gblks;
    p.tile0 = (uint32_t)tiles;
    gblks += rt;
    tiles += p.ly ? rt * ct : 0;
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
  gcdouble *fx = (gcdouble *)pr.fx + (uint64_t)r0 * 20;
  gdouble *g = (gdouble *)pr.g + (uint64_t)r0 * 20;
  for (uint32_t e = threadIdx.x; e < n; e += 256) sF[e] = fx[e];
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < n; e += 256) {
    const uint32_t x = e / 20u, j = e % 20u;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 20; i++) acc = fma(sF[x * 20 + i], sM[i * 20 + j], acc);
    g[e] = acc;
  }
}

// orders a wave's LDS accesses around its own tile
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One workgroup = 64 rows x 4 pieces of one pair (compact grid over all
// pairs' tiles); wave w takes piece p = 4 tc + w of every row.
//
// The stores are shaped for HBM.  Every store writes 64 consecutive scores
// of one row starting on a 128-byte line, so no line is written in parts by
// two stores: with s the first column of row x on a line boundary, piece p of
// the row is columns [64p + s - 16, 64p + s + 48) clipped to the row (the
// pieces tile the row; an extra piece finishes rows whose end lies past the
// last multiple of 64).  A wave computes the 80 columns 64p - 16 .. 64p + 63,
// which hold piece p of every row, and writes them row by row into its LDS
// tile; lane l then stores column lo + min(l, n) of the piece [lo, lo + n],
// so lanes past the piece repeat its last element, an empty piece repeats
// the row's last element, and rows past the end of the profile repeat its
// last row: every store is whole and writes only correct values.
//
// The matrix-core operands (fY of the 80 columns, G of the 64 rows) are
// loaded once, before the first store: inside the loop the wave issues only
// stores and LDS traffic, so no wait ever waits on its stores (a load after
// them would complete only after them).  Lane l supplies A[l%16][l/16] =
// G[row][4k + l/16] and B[l/16][l%16] = fY[col][4k + l/16] and holds
// D[l/16 + 4r][l%16] of each 16 x 16 block.
__global__ __launch_bounds__(256) void psp_scores_kernel(const PspWork *__restrict__ w, uint32_t npairs) {
  __shared__ double tiles[4][kPspRows][kPspSpan];
  const uint32_t q = pair_of(npairs, blockIdx.x, [&](uint32_t i) { return w[i].tile0; });
  const PspWork pr = w[q];
  const uint32_t lane = threadIdx.x & 63u, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t ly = pr.ly, npieces = psp_pieces(ly), nct = (npieces + kPspPieces - 1) / kPspPieces;
  const uint32_t t = blockIdx.x - pr.tile0;
  const uint32_t p = (t % nct) * kPspPieces + wave, xb = (t / nct) * kPspRowsPerTile;
  if (p >= npieces) return;
  const uint32_t li = lane & 15u, lk = lane >> 4;
  const int64_t yc = 64 * (int64_t)p - 16;  // first computed column (piece 0: columns -16 .. -1 unused)
  double b[5][5];
#pragma unroll
  for (int cb = 0; cb < 5; cb++) {  // columns outside the row: any valid column, never stored
    const uint32_t y = (uint32_t)min(max(yc + 16 * cb + li, (int64_t)0), (int64_t)ly - 1);
    gcdouble *fy = (gcdouble *)pr.fy + (uint64_t)y * 20 + lk;
#pragma unroll
    for (int k = 0; k < 5; k++) b[cb][k] = fy[4 * k];
  }
  double a[4][5];
#pragma unroll
  for (int rb = 0; rb < 4; rb++) {  // rows past the end: the last row
    const uint32_t x = min(xb + 16u * rb + li, pr.lx - 1u);
    gcdouble *g = (gcdouble *)pr.g + (uint64_t)x * 20 + lk;
#pragma unroll
    for (int k = 0; k < 5; k++) a[rb][k] = g[4 * k];
  }
  const uint64_t base8 = (uint64_t)(uintptr_t)pr.scores >> 3;  // address of S in doubles
  double(*tile)[kPspSpan] = tiles[wave];
#pragma unroll
  for (int rb = 0; rb < 4; rb++) {
    const uint32_t x0 = xb + 16u * rb;
    if (x0 >= pr.lx) break;
    v4d acc[5];
#pragma unroll
    for (int cb = 0; cb < 5; cb++) acc[cb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 5; k++)
#pragma unroll
      for (int cb = 0; cb < 5; cb++) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][k], b[cb][k], acc[cb], 0, 0, 0);
    wave_sync();  // the previous step's reads of the tile are done
#pragma unroll
    for (int cb = 0; cb < 5; cb++)
#pragma unroll
      for (int r = 0; r < 4; r++) tile[lk + 4 * r][16 * cb + li] = acc[cb][r];
    wave_sync();
#pragma unroll
    for (int h = 0; h < 2; h++) {
      double v[8];
      uint32_t off[8];
#pragma unroll
      for (int r = 0; r < 8; r++) {  // piece p of row x: [lo, lo + n]
        const uint32_t x = min(x0 + 8 * h + r, pr.lx - 1u);
        const uint32_t s = (16u - (uint32_t)((base8 + (uint64_t)x * ly) & 15u)) & 15u;
        const uint32_t lo0 = 64u * p + s > 16u ? 64u * p + s - 16u : 0u;
        const uint32_t hi = min(64u * p + s + 48u, ly);
        const uint32_t lo = lo0 < hi ? lo0 : ly - 1u;
        const uint32_t n = lo0 < hi ? hi - 1u - lo : 0u;
        const uint32_t d = min(lane, n);
        off[r] = lo + d;
        v[r] = tile[x - x0][(uint32_t)((int64_t)lo - yc) + d];
      }
#pragma unroll
      for (int r = 0; r < 8; r++) {
        gdouble *row = (gdouble *)pr.scores + (uint64_t)min(x0 + 8 * h + r, pr.lx - 1u) * ly;
        __builtin_nontemporal_store(v[r], row + off[r]);  // streamed: never read back here
      }
    }
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
