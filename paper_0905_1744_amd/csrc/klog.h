// Natural logarithm for the distance of Equation 2, d = -ln(Delta + F).
//
// Table-driven reduction after P. T. P. Tang, "Table-driven implementation
// of the logarithm function in IEEE floating-point arithmetic" (ACM TOMS
// 16(4), 1990): write x = m 2^e with m in [0.707, 1.414), pick the grid
// point c = 1 + j/128 nearest to m (|m - c| <= 1/256, so f = m - c is
// exact), and use ln x = e ln2 + ln c + ln(1 + r) with r = f / c, |r| <
// 0.0056.  ln(1 + r) is its Taylor series through r^6 (truncation below
// |r|^7 / 7 < 3e-17).  The 92 values 1/c and ln c, and ln 2, are computed
// at kernel start with correctly rounded division and the device's
// accurate log, so no constant is typed in.  Absolute error is a few 1e-16
// (plus |e| x 2e-17), far below what the 1e-12 rank tolerance needs, at
// about 20 instructions (one LDS read) instead of a general-purpose log.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace kd {

constexpr int kLogLo = -38;              // smallest j = round((m - 1) * 128)
constexpr int kLogEntries = 53 - kLogLo + 1;  // j in [-38, 53]

struct LogEntry {
  double inv_c;  // 1 / (1 + j/128)
  double ln_c;   // ln(1 + j/128)
};

__host__ __device__ inline void log_table_entry(int q, LogEntry &e) {
  const double c = 1.0 + (double)(q + kLogLo) * 0x1p-7;
  e.inv_c = 1.0 / c;
  e.ln_c = log(c);
}

// x must be positive and normal; kNeg returns -ln x (the same bits negated).
// The fold: m in [0.70703125, 1.4140625), so the nearest grid point is
// 1 + j/128 with j in [-38, 53].  The exponent comes from the high word of
// the bit pattern: less the high word of 0.70703125 (0x3FE6A000), its top
// twelve bits are e, and removing them from x's exponent field leaves m.
template <bool kNeg = false>
__host__ __device__ __forceinline__ double log_tab(double x, const LogEntry *tab, double ln2) {
  const unsigned long long bx = __builtin_bit_cast(unsigned long long, x);
  const uint32_t lo = (uint32_t)bx, hi = (uint32_t)(bx >> 32);
  const uint32_t th = hi - 0x3FE6A000u;
  const int e = (int)th >> 20;
  const double m = __builtin_bit_cast(double, ((unsigned long long)(hi - (th & 0xFFF00000u)) << 32) | lo);
  const double jd = rint((m - 1.0) * 128.0);  // exact before rounding
  const int j = (int)jd;
  const double f = m - fma(jd, 0x1p-7, 1.0);      // exact: |m - c| <= 1/256
  const LogEntry t = tab[j - kLogLo];
  const double r = f * t.inv_c;
  double p = fma(r, -1.0 / 6.0, 0.2);
  p = fma(r, p, -0.25);
  p = fma(r, p, 1.0 / 3.0);
  p = fma(r, p, -0.5);
  p = fma(r, p, 1.0);
  // e ln2 + ln c + r p; negating every operand negates the rounded result
  const double sg = kNeg ? -1.0 : 1.0;
  return fma(sg * (double)e, ln2, fma(sg * r, p, sg * t.ln_c));
}
}  // namespace kd
