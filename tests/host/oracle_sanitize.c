/*
 * Drives every entry point of the CPU oracle (oracle/kd_oracle.c) on small
 * seeded inputs, including the edge cases its callers reach (the shortest
 * and the longest sequence, bad residues, one bucket, B = N, one-leaf and
 * tied trees, empty profiles), so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer sees every code path.  Test infrastructure:
 * built and run by tests/test_host_helpers.py on the CPU.  Exit status 0 and
 * the line "OK" mean no sanitizer report and every checked value right.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_code(uint8_t ch);
int64_t orc_kmer_words(const uint8_t *s, uint64_t n, uint32_t *words, uint64_t *bad_pos);
int64_t orc_count_dense(const uint8_t *s, uint64_t n, uint32_t *dense);
int orc_count_set(const uint8_t *res, const uint64_t *offsets, uint32_t N, uint16_t *ids,
                  uint16_t *cnt, uint64_t *off, uint32_t *K, uint64_t *err_seq, uint64_t *err_pos);
uint32_t orc_shared(const uint16_t *ia, const uint16_t *ca, uint64_t na, const uint16_t *ib,
                    const uint16_t *cb, uint64_t nb);
uint32_t orc_shared_dense(const uint32_t *cx, const uint32_t *cy);
double orc_fraction(uint32_t shared, uint32_t denom);
double orc_distance(double F, double delta);
void orc_similarity_block(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                          const uint32_t *K, uint32_t r0, uint32_t nr, uint32_t c0, uint32_t nc,
                          uint16_t *shared, uint16_t *denom);
void orc_rank_rows(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off, const uint32_t *K,
                   uint32_t N, const uint32_t *rows, uint32_t nrows, double delta, double *out,
                   double *scale);
int orc_partition(const double *R, uint32_t N, uint32_t B, uint32_t *bucket, uint32_t *order,
                  uint32_t *offsets, double *piv_r, uint32_t *piv_i);
int orc_local_ranks(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off, const uint32_t *K,
                    uint32_t N, uint32_t B, double delta, double *out);
int orc_global_samples(const double *local, uint32_t N, uint32_t B, uint32_t k, uint32_t *samples);
void orc_global_rank_rows(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                          const uint32_t *K, const uint32_t *samples, uint32_t S,
                          const uint32_t *rows, uint32_t nrows, double delta, double *out,
                          double *scale);
void orc_distance_block(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                        const uint32_t *K, const uint32_t *rows, uint32_t nr, const uint32_t *cols,
                        uint32_t nc, double delta, double *out);
int orc_upgma(const double *d, uint32_t n, int32_t *merges, double *heights);
int orc_profile(const uint8_t *aln, uint32_t m, uint32_t L, double *f, uint64_t *bad);
void orc_psp(const double *fx, uint32_t Lx, const double *fy, uint32_t Ly, const double *M, double *S);
int orc_psp_matrix(const double *P, double *M);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void) { /* xorshift64* (Vigna) */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int failures = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      failures++;                                                    \
    }                                                                \
  } while (0)

static const char AA[] = "ACDEFGHIKLMNPQRSTVWY";

/* A set of N random sequences over the first `na` amino acids, lengths in
 * [lmin, lmax]; the residues are allocated to their exact size. */
static uint8_t *make_set(uint32_t N, uint32_t lmin, uint32_t lmax, int na, uint64_t *off) {
  off[0] = 0;
  for (uint32_t i = 0; i < N; i++) off[i + 1] = off[i] + lmin + next_u32() % (lmax - lmin + 1);
  uint8_t *res = (uint8_t *)malloc(off[N]);
  for (uint64_t t = 0; t < off[N]; t++) res[t] = (uint8_t)AA[next_u32() % (uint32_t)na];
  return res;
}

static void run_set(uint32_t N, uint32_t lmin, uint32_t lmax, int na, uint32_t B, double delta) {
  uint64_t *off_in = (uint64_t *)malloc(sizeof(uint64_t) * (N + 1));
  uint8_t *res = make_set(N, lmin, lmax, na, off_in);
  uint64_t cap = off_in[N] - 5ull * N;
  uint16_t *ids = (uint16_t *)malloc(2 * cap), *cnt = (uint16_t *)malloc(2 * cap);
  uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (N + 1));
  uint32_t *K = (uint32_t *)malloc(4ull * N);
  uint64_t es = 0, ep = 0;
  CHECK(orc_count_set(res, off_in, N, ids, cnt, off, K, &es, &ep) == 0);
  for (uint32_t i = 0; i < N; i++) CHECK(K[i] == off_in[i + 1] - off_in[i] - 5);

  /* dense route for the first two sequences */
  uint32_t *cx = (uint32_t *)calloc(46656, 4), *cy = (uint32_t *)calloc(46656, 4);
  CHECK(orc_count_dense(res, off_in[1], cx) == (int64_t)K[0]);
  CHECK(orc_count_dense(res + off_in[1], off_in[2] - off_in[1], cy) == (int64_t)K[1]);
  const uint32_t s01 = orc_shared(ids + off[0], cnt + off[0], off[1] - off[0], ids + off[1],
                                  cnt + off[1], off[2] - off[1]);
  CHECK(orc_shared_dense(cx, cy) == s01);

  /* a block away from the origin, and the full square */
  const uint32_t r0 = N / 3, nr = N - r0, c0 = N / 2, nc = N - c0;
  uint16_t *S = (uint16_t *)malloc(2ull * nr * nc), *D = (uint16_t *)malloc(2ull * nr * nc);
  orc_similarity_block(ids, cnt, off, K, r0, nr, c0, nc, S, D);
  orc_similarity_block(ids, cnt, off, K, r0, nr, c0, nc, S, NULL);

  uint32_t *rows = (uint32_t *)malloc(4ull * N);
  for (uint32_t i = 0; i < N; i++) rows[i] = N - 1 - i;
  double *R = (double *)malloc(8ull * N), *sc = (double *)malloc(8ull * N);
  orc_rank_rows(ids, cnt, off, K, N, rows, N, delta, R, sc);
  orc_rank_rows(ids, cnt, off, K, N, rows, 1, delta, R, NULL);
  for (uint32_t i = 0; i < N; i++) CHECK(R[i] >= -log1p(delta) - 1e-12 && R[i] <= -log(delta) + 1e-12);

  uint32_t *bucket = (uint32_t *)malloc(4ull * N), *order = (uint32_t *)malloc(4ull * N);
  uint32_t *offs = (uint32_t *)malloc(4ull * (N + 1));
  double *pr = (double *)malloc(8ull * (N + 1));
  uint32_t *pi = (uint32_t *)malloc(4ull * (N + 1));
  const uint32_t Bs[] = {1, B, N};
  for (int q = 0; q < 3; q++) {
    CHECK(orc_partition(R, N, Bs[q], bucket, order, offs, pr, pi) == 0);
    CHECK(offs[0] == 0 && offs[Bs[q]] == N);
    CHECK(orc_partition(R, N, Bs[q], bucket, order, offs, NULL, NULL) == 0);
  }
  CHECK(orc_partition(R, N, 0, bucket, order, offs, pr, pi) != 0);
  CHECK(orc_partition(R, N, N + 1, bucket, order, offs, pr, pi) != 0);

  double *loc = (double *)malloc(8ull * N);
  CHECK(orc_local_ranks(ids, cnt, off, K, N, B, delta, loc) == 0);
  CHECK(orc_local_ranks(ids, cnt, off, K, N, N + 1, delta, loc) != 0);
  const uint32_t k = N / B;
  uint32_t *smp = (uint32_t *)malloc(4ull * B * k);
  CHECK(orc_global_samples(loc, N, B, k, smp) == 0);
  CHECK(orc_global_samples(loc, N, B, k + N, smp) != 0);
  CHECK(orc_global_samples(loc, N, B, 0, smp) != 0);
  orc_global_rank_rows(ids, cnt, off, K, smp, B * k, rows, N, delta, R, sc);
  orc_global_rank_rows(ids, cnt, off, K, smp, B * k, rows, 2, delta, R, NULL);

  const uint32_t n = N < 40 ? N : 40;
  double *dm = (double *)malloc(8ull * n * n);
  orc_distance_block(ids, cnt, off, K, rows, n, rows, n, delta, dm);
  int32_t *merges = (int32_t *)malloc(8ull * n);
  double *h = (double *)malloc(8ull * n);
  CHECK(orc_upgma(dm, n, merges, h) == 0);
  for (uint32_t t = 0; t + 1 < n; t++) CHECK(merges[2 * t] < merges[2 * t + 1]);

  free(res); free(off_in); free(ids); free(cnt); free(off); free(K); free(cx); free(cy);
  free(S); free(D); free(rows); free(R); free(sc); free(bucket); free(order); free(offs);
  free(pr); free(pi); free(loc); free(smp); free(dm); free(merges); free(h);
}

static void run_edges(void) {
  /* shortest and longest sequences, and every error */
  uint32_t w[8];
  uint64_t bad = 0;
  CHECK(orc_kmer_words((const uint8_t *)"ACDEF", 5, w, &bad) < 0);
  CHECK(orc_kmer_words((const uint8_t *)"ACDEFG", 6, w, &bad) == 1);
  CHECK(orc_kmer_words((const uint8_t *)"ACDXFGH", 7, w, &bad) < 0 && bad == 3);
  const uint64_t nmax = 65535 + 5;
  uint8_t *lng = (uint8_t *)malloc(nmax + 1);
  memset(lng, 'A', nmax + 1);
  uint32_t *words = (uint32_t *)malloc(4 * (nmax + 1));
  CHECK(orc_kmer_words(lng, nmax, words, &bad) == 65535);
  CHECK(orc_kmer_words(lng, nmax + 1, words, &bad) < 0);
  uint32_t *dense = (uint32_t *)calloc(46656, 4);
  CHECK(orc_count_dense(lng, nmax, dense) == 65535 && dense[0] == 65535);
  uint64_t off_in[3] = {0, 6, 6 + nmax};
  uint8_t *res = (uint8_t *)malloc(off_in[2]);
  memcpy(res, "CCCCCC", 6);
  memset(res + 6, 'A', nmax);
  uint16_t *ids = (uint16_t *)malloc(2 * 65536), *cnt = (uint16_t *)malloc(2 * 65536);
  uint64_t off[3];
  uint32_t K[2];
  uint64_t es = 0, ep = 0;
  CHECK(orc_count_set(res, off_in, 2, ids, cnt, off, K, &es, &ep) == 0);
  CHECK(K[0] == 1 && K[1] == 65535 && ids[0] == 9331 && cnt[1] == 65535);
  res[7] = 'X';
  CHECK(orc_count_set(res, off_in, 2, ids, cnt, off, K, &es, &ep) == -2 && es == 1 && ep == 1);
  CHECK(orc_fraction(7, 7) == 1.0 && orc_distance(0.75, 0.25) == 0.0);
  CHECK(orc_code('B') < 0 && orc_code('V') == 5);

  /* trees: one leaf, all-equal ties, zero leaves refused */
  double d1 = 0.0;
  int32_t mg[64];
  double ht[32];
  CHECK(orc_upgma(&d1, 1, mg, ht) == 0);
  CHECK(orc_upgma(&d1, 0, mg, ht) != 0);
  double eq[25];
  for (int q = 0; q < 25; q++) eq[q] = 1.0;
  CHECK(orc_upgma(eq, 5, mg, ht) == 0 && mg[0] == 0 && mg[1] == 1);

  /* profiles and PSP: empty, gaps, a bad byte; the log-odds matrix */
  double f[20 * 8], g[20 * 8], Ssc[64], M[400], P[400];
  const uint8_t aln[] = "AC-D.EFG" "WWWWWWWW";
  CHECK(orc_profile(aln, 2, 8, f, &bad) == 0);
  CHECK(orc_profile(aln, 2, 0, f, &bad) == 0);
  CHECK(orc_profile(aln, 0, 8, f, &bad) != 0);
  const uint8_t badaln[] = "ACZD";
  CHECK(orc_profile(badaln, 1, 4, g, &bad) == -2 && bad == 2);
  double tot = 0.0;
  for (int q = 0; q < 400; q++) tot += (P[q] = 1.0 + (double)(next_u32() % 100));
  for (int q = 0; q < 400; q++) P[q] /= tot;
  CHECK(orc_psp_matrix(P, M) == 0);
  P[7] = 0.0;
  CHECK(orc_psp_matrix(P, M) != 0);
  CHECK(orc_profile(aln, 2, 8, g, &bad) == 0);
  orc_psp(f, 8, g, 8, M, Ssc);
  orc_psp(f, 0, g, 8, M, Ssc);
  free(lng); free(words); free(dense); free(res); free(ids); free(cnt);
}

int main(void) {
  run_edges();
  run_set(37, 6, 60, 20, 4, 0.1);   /* tiny sequences, many empty pairs */
  run_set(64, 30, 200, 3, 8, 0.01); /* three letters: repeated words, counts >= 2 */
  run_set(100, 50, 400, 20, 10, 0.5);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("OK\n");
  return 0;
}
