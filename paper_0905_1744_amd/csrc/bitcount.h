// Bit-sliced counting used by the all-pairs kernels.
//
// A 32-bit word holds 32 independent one-bit counter inputs.  Words are
// summed with carry-save adders (the Harley-Seal scheme: a tree of
// full adders whose carries move to the next weight) into bit planes: bit q
// of plane P[k] is bit k of counter q.  P[0..3] are the adder tree's state
// (weights 1, 2, 4, 8); every 16 input words the tree emits one word of
// weight 16 that is rippled into P[4..NP).  NP = planes needed for the
// largest count a counter can reach.
//
// transpose16 turns the 16 planes into 16 counters per half-word: on exit
// A[r] holds counter r in bits 0..15 and counter 16+r in bits 16..31.
//
// Everything here is plain integer logic, usable on the host for checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kd {

// Three-input parity and majority.  On gfx950 each is one v_bitop3_b32
// whose 8-bit immediate is the function's truth table evaluated on the
// operand masks 0xF0, 0xCC, 0xAA (parity 0x96, majority 0xE8; both
// functions are symmetric, so operand order does not matter).  The host
// pass (used only by the CPU checks) spells them out.
__host__ __device__ __forceinline__ uint32_t parity3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

__host__ __device__ __forceinline__ uint32_t majority3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
#else
  return (a & b) | (a & c) | (b & c);
#endif
}

// (hi, lo) <- carry and sum of the full adder (lo, a, b)
__host__ __device__ __forceinline__ void csa(uint32_t &hi, uint32_t &lo, uint32_t a, uint32_t b) {
  const uint32_t x = lo;
  hi = majority3(x, a, b);
  lo = parity3(x, a, b);
}

template <int NP>
__host__ __device__ __forceinline__ void ripple(uint32_t (&P)[16], uint32_t c, int from) {
#pragma unroll
  for (int k = 0; k < NP; k++) {
    if (k >= from) {
      const uint32_t t = P[k] & c;
      P[k] ^= c;
      c = t;
    }
  }
}

// adds 16 words
template <int NP>
__host__ __device__ __forceinline__ void add16(uint32_t (&P)[16], const uint32_t (&w)[16]) {
  uint32_t tA, tB, fA, fB, eA, eB, s16;
  csa(tA, P[0], w[0], w[1]);
  csa(tB, P[0], w[2], w[3]);
  csa(fA, P[1], tA, tB);
  csa(tA, P[0], w[4], w[5]);
  csa(tB, P[0], w[6], w[7]);
  csa(fB, P[1], tA, tB);
  csa(eA, P[2], fA, fB);
  csa(tA, P[0], w[8], w[9]);
  csa(tB, P[0], w[10], w[11]);
  csa(fA, P[1], tA, tB);
  csa(tA, P[0], w[12], w[13]);
  csa(tB, P[0], w[14], w[15]);
  csa(fB, P[1], tA, tB);
  csa(eB, P[2], fA, fB);
  csa(s16, P[3], eA, eB);
  ripple<NP>(P, s16, 4);
}

// adds 8 words (the tail of a list whose length is 16 mod 32)
template <int NP>
__host__ __device__ __forceinline__ void add8(uint32_t (&P)[16], const uint32_t (&w)[8]) {
  uint32_t tA, tB, fA, fB, e8;
  csa(tA, P[0], w[0], w[1]);
  csa(tB, P[0], w[2], w[3]);
  csa(fA, P[1], tA, tB);
  csa(tA, P[0], w[4], w[5]);
  csa(tB, P[0], w[6], w[7]);
  csa(fB, P[1], tA, tB);
  csa(e8, P[2], fA, fB);
  ripple<NP>(P, e8, 3);
}

__host__ __device__ __forceinline__ void swap_bits(uint32_t &x, uint32_t &y, int j, uint32_t m) {
  const uint32_t t = ((x >> j) ^ y) & m;
  y ^= t;
  x ^= t << j;
}

// Two 16x16 bit-matrix transposes, one per half-word: bit (16h + r) of A[k]
// on entry is bit (16h + k) of A[r] on exit.
__host__ __device__ __forceinline__ void transpose16(uint32_t (&A)[16]) {
#pragma unroll
  for (int k = 0; k < 8; k++) swap_bits(A[k], A[k + 8], 8, 0x00FF00FFu);
#pragma unroll
  for (int k = 0; k < 16; k++)
    if (!(k & 4)) swap_bits(A[k], A[k + 4], 4, 0x0F0F0F0Fu);
#pragma unroll
  for (int k = 0; k < 16; k++)
    if (!(k & 2)) swap_bits(A[k], A[k + 2], 2, 0x33333333u);
#pragma unroll
  for (int k = 0; k < 16; k += 2) swap_bits(A[k], A[k + 1], 1, 0x55555555u);
}

// planes needed when each counter sees at most `words` inputs
__host__ __device__ __forceinline__ int planes_for(uint32_t words) {
  int b = 0;
  while (b < 32 && (words >> b)) b++;
  return b;
}

}  // namespace kd
