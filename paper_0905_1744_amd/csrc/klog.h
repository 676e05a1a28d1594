// Natural logarithm for the distance of Equation 2, d = -ln(Delta + F).
//
// Table-driven reduction after P. T. P. Tang, "Table-driven implementation
// of the logarithm function in IEEE floating-point arithmetic" (ACM TOMS
// 16(4), 1990): write x = m 2^e with m in [0.707, 1.414), pick the grid
// point c = 1 + j/128 nearest to m (|m - c| <= 1/256, so f = m - c is
// exact), and use ln x = e ln2 + ln c + ln(1 + r) with r = f / c, |r| <=
// 2^-8.  ln(1 + r) is its Taylor series through r^6 (truncation below
// |r|^7 / 7 < 3e-18).  The 92 values 1/c and ln c, and ln 2, are computed
// at kernel start with correctly rounded division and the device's
// accurate log, so no constant is typed in.  Absolute error is a few 1e-16
// (plus |e| x 2e-17), far below what the 1e-12 rank tolerance needs, at
// about 16 instructions instead of a general-purpose log.
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

// x must be positive and normal
__host__ __device__ __forceinline__ double log_tab(double x, const LogEntry *tab, double ln2) {
  int e;
  double m = frexp(x, &e);  // [0.5, 1)
  m *= 2.0;
  e -= 1;                   // [1, 2)
  if (m > 1.4140625) {      // fold into [0.707, 1.414)
    m *= 0.5;
    e += 1;
  }
  const double jd = rint((m - 1.0) * 128.0);
  const int j = (int)jd;
  const double f = m - (1.0 + jd * 0x1p-7);
  const LogEntry t = tab[j - kLogLo];
  const double r = f * t.inv_c;
  double p = fma(r, -1.0 / 6.0, 0.2);
  p = fma(r, p, -0.25);
  p = fma(r, p, 1.0 / 3.0);
  p = fma(r, p, -0.5);
  p = fma(r, p, 1.0);
  p *= r;
  return fma((double)e, ln2, t.ln_c + p);
}

}  // namespace kd
