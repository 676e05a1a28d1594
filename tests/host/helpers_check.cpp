// Host-side checks of device helpers that are plain arithmetic: the
// table-driven log against the C library's log, and the bit-sliced
// carry-save counting + plane transpose against direct counting.
// Built with hipcc as host code by tests/test_host_helpers.py.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>

#include "bitcount.h"
#include "klog.h"

using namespace kd;

static int check_log() {
  LogEntry tab[kLogEntries];
  for (int q = 0; q < kLogEntries; q++) log_table_entry(q, tab[q]);
  const double ln2 = log(2.0);
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  double worst = 0, worst_x = 0;
  long n = 0;
  auto one = [&](double x) {
    const double a = log_tab(x, tab, ln2), b = log(x);
    const double err = fabs(a - b) / fmax(1.0, fabs(b));
    if (err > worst) { worst = err; worst_x = x; }
    n++;
  };
  for (int i = 0; i < 2000000; i++) one(0.1 + 1.0 * u(g));           // Delta = 0.1 range
  for (int i = 0; i < 200000; i++) one(ldexp(1.0 + u(g), -(int)(u(g) * 1000)));  // down to 2^-1000
  for (int i = 0; i < 200000; i++) one(1.0 + (u(g) - 0.5) * 1e-6);    // near 1
  for (int k = 1; k <= 65535; k += 7)                                // exact fractions S/D + 0.1
    for (int s = 0; s <= k; s += 1 + k / 50) one(0.1 + (double)s / (double)k);
  printf("log: %ld points, worst scaled error %.3g at x=%.17g\n", n, worst, worst_x);
  return worst <= 1e-15 ? 0 : 1;
}

template <int NP>
static int check_count_np(std::mt19937_64 &g, int L) {
  // L ids of one lane: masks m[t] (16 bits, row r set) ; words = m[2i] | m[2i+1] << 16
  uint32_t P[16] = {0};
  int direct[32] = {0};
  uint16_t *m = new uint16_t[L];
  for (int t = 0; t < L; t++) {
    m[t] = (uint16_t)(g() & 0xFFFF);
    if ((g() & 3) == 0) m[t] = 0xFFFF;  // saturating runs
    for (int r = 0; r < 16; r++) direct[(t & 1) * 16 + r] += (m[t] >> r) & 1;
  }
  int t = 0;
  for (; t + 32 <= L; t += 32) {
    uint32_t w[16];
    for (int i = 0; i < 16; i++) w[i] = m[t + 2 * i] | ((uint32_t)m[t + 2 * i + 1] << 16);
    add16<NP>(P, w);
  }
  if (t < L) {  // L % 32 == 16
    uint32_t w[8];
    for (int i = 0; i < 8; i++) w[i] = m[t + 2 * i] | ((uint32_t)m[t + 2 * i + 1] << 16);
    add8<NP>(P, w);
  }
  transpose16(P);
  int bad = 0;
  for (int r = 0; r < 16; r++) {
    const int lo = P[r] & 0xFFFF, hi = P[r] >> 16;
    if (lo != direct[r] || hi != direct[16 + r]) bad++;
  }
  delete[] m;
  return bad;
}

static int check_count() {
  std::mt19937_64 g(11);
  int bad = 0, cases = 0;
  for (int L = 16; L <= 65536; L = (L < 1024 ? L + 16 : L * 2)) {
    const int need = planes_for((uint32_t)(L / 2));
    int b;
    if (need <= 8) b = check_count_np<8>(g, L);
    else if (need <= 10) b = check_count_np<10>(g, L);
    else if (need <= 12) b = check_count_np<12>(g, L);
    else if (need <= 14) b = check_count_np<14>(g, L);
    else b = check_count_np<16>(g, L);
    bad += b;
    cases++;
  }
  printf("bit-sliced counting: %d list lengths, %d wrong counters\n", cases, bad);
  return bad ? 1 : 0;
}

int main() {
  int rc = check_log();
  rc |= check_count();
  printf(rc ? "FAIL\n" : "OK\n");
  return rc;
}
