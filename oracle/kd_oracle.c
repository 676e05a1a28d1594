/*
 * CPU oracle for the k-mer rank + regular-sampling decomposition front end of
 * Sample-Align-D (Saeed & Khokhar, "A Domain Decomposition Strategy for
 * Alignment of Multiple Biological Sequences on Multiprocessor Platforms").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness authority that the
 * GPU library is compared against.  Only the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or constant with the GPU library.
 *
 * Plain, single-threaded, obviously-correct C.  Every function follows the
 * paper's definitions in the paper's order:
 *
 *   k-mer words and count vectors ........ Section 3, "k-mer Rank" paragraph
 *   common count C_i = min(cX_i, cY_i) ... Section 3 (same paragraph)
 *   fraction F(X,Y) ...................... Equation 1
 *   distance d = -log(Delta + F) ......... Equation 2
 *   k-mer rank R_i = (1/N) sum_j d(i,j) .. Equation 3
 *   local sort, regular samples, pivots,
 *   bucket assignment .................... Section 3.1.2 ("Redistribution
 *                                          Based on Globalized k-mer Rank"),
 *                                          Algorithm 2 steps 3 and 8-11
 *   local ranks, k samples per processor,
 *   globalized rank ...................... Section 3.1.1 ("Globalised k-mer
 *                                          Rank"), Algorithm 2 steps 1-6
 *   profile of an alignment, PSP score ... Section 3.1.3, Equation 4
 *   per-bucket distance matrix and
 *   guide tree ........................... Section 2 (the generic scheme: a
 *                                          pairwise similarity matrix, then
 *                                          a guide tree) applied to each
 *                                          bucket (Section 3.1.3); the tree
 *                                          is UPGMA (average linkage)
 *
 * Readings where the paper is silent (alphabet, k, Delta, log base, sample
 * positions, pivot indices for odd p, ties) are fixed by the caller-visible
 * parameters described next to each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_K 6            /* k-mer length used by every workload */
#define ORC_C 6            /* Dayhoff-6 alphabet size c */
#define ORC_EPS 46656      /* epsilon = c^k distinct words */

#define ORC_OK 0
#define ORC_EBADRESIDUE (-2)
#define ORC_ESHORTSEQ (-3)
#define ORC_ETOOLONG (-4)
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-5)

/* Dayhoff-6 grouping of the 20 standard amino acids:
 * {A,G,P,S,T} {C} {D,E,N,Q} {F,W,Y} {H,K,R} {I,L,M,V} -> 0..5.
 * Any other byte is not a residue of the alphabet. */
int orc_code(uint8_t ch)
{
    switch (ch) {
    case 'A': case 'G': case 'P': case 'S': case 'T': return 0;
    case 'C': return 1;
    case 'D': case 'E': case 'N': case 'Q': return 2;
    case 'F': case 'W': case 'Y': return 3;
    case 'H': case 'K': case 'R': return 4;
    case 'I': case 'L': case 'M': case 'V': return 5;
    default: return -1;
    }
}

/* The n-k+1 k-mer words of X in position order.  Word t is the base-c
 * number whose most significant digit is residue t (big-endian).  Returns
 * the number of words K = n-k+1, or a negative error with *bad_pos set. */
int64_t orc_kmer_words(const uint8_t *s, uint64_t n, uint32_t *words, uint64_t *bad_pos)
{
    if (n < ORC_K) { if (bad_pos) *bad_pos = 0; return ORC_ESHORTSEQ; }
    if (n - ORC_K + 1 > 65535) { if (bad_pos) *bad_pos = 0; return ORC_ETOOLONG; }
    for (uint64_t t = 0; t < n; t++)
        if (orc_code(s[t]) < 0) { if (bad_pos) *bad_pos = t; return ORC_EBADRESIDUE; }
    uint64_t K = n - ORC_K + 1;
    for (uint64_t t = 0; t < K; t++) {
        uint32_t w = 0;
        for (int u = 0; u < ORC_K; u++)
            w = w * ORC_C + (uint32_t)orc_code(s[t + u]);
        words[t] = w;
    }
    return (int64_t)K;
}

/* Count vector c^X over all epsilon words (Section 3): dense[w] = number of
 * occurrences of word w in X.  Returns K or a negative error. */
int64_t orc_count_dense(const uint8_t *s, uint64_t n, uint32_t *dense)
{
    uint64_t K = n >= ORC_K ? n - ORC_K + 1 : 1;
    uint32_t *w = (uint32_t *)malloc(sizeof(uint32_t) * (K ? K : 1));
    if (!w) return ORC_ENOMEM;
    int64_t r = orc_kmer_words(s, n, w, NULL);
    if (r >= 0) {
        memset(dense, 0, sizeof(uint32_t) * ORC_EPS);
        for (int64_t t = 0; t < r; t++) dense[w[t]]++;
    }
    free(w);
    return r;
}

/* Count vectors of a whole set, stored as the nonzero entries of each c^X in
 * increasing word order: (ids[j], cnt[j]) for j in off[i]..off[i+1).  The
 * caller sizes ids/cnt for sum_i (n_i - k + 1) entries.  K[i] = n_i - k + 1.
 * On error returns the negative code with *err_seq / *err_pos set. */
int orc_count_set(const uint8_t *res, const uint64_t *offsets, uint32_t N,
                  uint16_t *ids, uint16_t *cnt, uint64_t *off, uint32_t *K,
                  uint64_t *err_seq, uint64_t *err_pos)
{
    uint32_t *dense = (uint32_t *)malloc(sizeof(uint32_t) * ORC_EPS);
    if (!dense) return ORC_ENOMEM;
    uint64_t o = 0;
    off[0] = 0;
    for (uint32_t i = 0; i < N; i++) {
        uint64_t n = offsets[i + 1] - offsets[i];
        uint32_t *w = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
        if (!w) { free(dense); return ORC_ENOMEM; }
        uint64_t bad = 0;
        int64_t r = orc_kmer_words(res + offsets[i], n, w, &bad);
        if (r < 0) {
            free(w); free(dense);
            if (err_seq) *err_seq = i;
            if (err_pos) *err_pos = bad;
            return (int)r;
        }
        memset(dense, 0, sizeof(uint32_t) * ORC_EPS);
        for (int64_t t = 0; t < r; t++) dense[w[t]]++;
        free(w);
        for (uint32_t x = 0; x < ORC_EPS; x++) {
            if (dense[x]) { ids[o] = (uint16_t)x; cnt[o] = (uint16_t)dense[x]; o++; }
        }
        off[i + 1] = o;
        K[i] = (uint32_t)r;
    }
    free(dense);
    return ORC_OK;
}

/* Common k-mer count sum_w min(c^X_w, c^Y_w) (Section 3; the paper's
 * min(c^X_i, c^Y_j) is read as the same word i on both sides).  Words absent
 * from either vector contribute min(.,0) = 0, so only words present in both
 * sorted entry lists are visited. */
uint32_t orc_shared(const uint16_t *ia, const uint16_t *ca, uint64_t na,
                    const uint16_t *ib, const uint16_t *cb, uint64_t nb)
{
    uint64_t a = 0, b = 0;
    uint32_t s = 0;
    while (a < na && b < nb) {
        if (ia[a] < ib[b]) a++;
        else if (ia[a] > ib[b]) b++;
        else { s += ca[a] < cb[b] ? ca[a] : cb[b]; a++; b++; }
    }
    return s;
}

/* Same quantity straight from two dense count vectors (literal sum over all
 * epsilon words). */
uint32_t orc_shared_dense(const uint32_t *cx, const uint32_t *cy)
{
    uint32_t s = 0;
    for (uint32_t w = 0; w < ORC_EPS; w++) s += cx[w] < cy[w] ? cx[w] : cy[w];
    return s;
}

/* Equation 1: F = shared / (min(n, m) - k + 1), in IEEE double. */
double orc_fraction(uint32_t shared, uint32_t denom)
{
    return (double)shared / (double)denom;
}

/* Equation 2: d = -log(Delta + F) with the natural logarithm. */
double orc_distance(double F, double delta)
{
    return -log(delta + F);
}

/* Shared counts and denominators for the block of rows r0..r0+nr-1 against
 * columns c0..c0+nc-1 (row-major nr x nc). denom may be NULL. */
void orc_similarity_block(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                          const uint32_t *K, uint32_t r0, uint32_t nr, uint32_t c0, uint32_t nc,
                          uint16_t *shared, uint16_t *denom)
{
    for (uint32_t r = 0; r < nr; r++) {
        uint32_t i = r0 + r;
        for (uint32_t c = 0; c < nc; c++) {
            uint32_t j = c0 + c;
            uint32_t s = orc_shared(ids + off[i], cnt + off[i], off[i + 1] - off[i],
                                    ids + off[j], cnt + off[j], off[j + 1] - off[j]);
            shared[(uint64_t)r * nc + c] = (uint16_t)s;
            if (denom) denom[(uint64_t)r * nc + c] = (uint16_t)(K[i] < K[j] ? K[i] : K[j]);
        }
    }
}

/* Equation 3 for the listed rows: R_i = (1/N) sum_{j=1..N} d(F(i,j)), the
 * sum running over every j including i itself, in increasing j, with
 * Neumaier-compensated addition so that the oracle's own rounding stays far
 * below the comparison tolerance. */
void orc_rank_rows(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                   const uint32_t *K, uint32_t N, const uint32_t *rows, uint32_t nrows,
                   double delta, double *out, double *scale)
{
    for (uint32_t q = 0; q < nrows; q++) {
        uint32_t i = rows[q];
        double sum = 0.0, comp = 0.0, mag = 0.0;
        for (uint32_t j = 0; j < N; j++) {
            uint32_t s = orc_shared(ids + off[i], cnt + off[i], off[i + 1] - off[i],
                                    ids + off[j], cnt + off[j], off[j + 1] - off[j]);
            uint32_t D = K[i] < K[j] ? K[i] : K[j];
            double d = orc_distance(orc_fraction(s, D), delta);
            double t = sum + d;
            if (fabs(sum) >= fabs(d)) comp += (sum - t) + d;
            else comp += (d - t) + sum;
            sum = t;
            mag += fabs(d);
        }
        out[q] = (sum + comp) / (double)N;
        /* (1/N) sum_j |d(i,j)|: the magnitude a comparison tolerance scales with */
        if (scale) scale[q] = mag / (double)N;
    }
}

/* ---- regular-sampling decomposition (Section 3.1.2, Algorithm 2) ---- */

typedef struct { double r; uint32_t i; } orc_key;

/* Keys are (rank, sequence index) compared lexicographically, so that equal
 * ranks are ordered by index and every key is distinct. */
static int orc_key_cmp(const void *pa, const void *pb)
{
    const orc_key *a = (const orc_key *)pa, *b = (const orc_key *)pb;
    if (a->r < b->r) return -1;
    if (a->r > b->r) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

static int orc_key_lt(orc_key a, orc_key b) { return orc_key_cmp(&a, &b) < 0; }

/* Split N ranked sequences into B buckets as the paper's p processors would:
 *  1. processor b holds the contiguous input block [floor(bN/B), floor((b+1)N/B))
 *     and sorts it by key (Algorithm 2 step 3 / step 7);
 *  2. from each sorted block of w_b keys it takes B-1 evenly spaced samples,
 *     the keys at 0-based positions floor(t*w_b/B), t = 1..B-1 (step 8);
 *  3. the B(B-1) samples are sorted and the keys at the paper's 1-based
 *     positions (i-1)B + B/2 (B/2 rounded down), i = 1..B-1, become the pivots
 *     (step 9);
 *  4. a key goes to bucket b when it lies in (pivot_{b-1}, pivot_b], i.e.
 *     bucket = number of pivots strictly below the key (step 11).
 * Outputs: bucket[N]; order[N] = indices grouped by bucket, each bucket in
 * key order; offsets[B+1] = bucket boundaries in order[]; pivot rank/index
 * arrays of B-1 entries (either may be NULL). */
int orc_partition(const double *R, uint32_t N, uint32_t B, uint32_t *bucket, uint32_t *order,
                  uint32_t *offsets, double *piv_r, uint32_t *piv_i)
{
    if (N == 0 || B == 0 || B > N) return ORC_EINVAL;
    orc_key *blk = (orc_key *)malloc(sizeof(orc_key) * N);
    orc_key *smp = (orc_key *)malloc(sizeof(orc_key) * ((size_t)B * (B - 1) + 1));
    orc_key *piv = (orc_key *)malloc(sizeof(orc_key) * (B ? B : 1));
    uint32_t *fill = (uint32_t *)calloc(B + 1, sizeof(uint32_t));
    if (!blk || !smp || !piv || !fill) { free(blk); free(smp); free(piv); free(fill); return ORC_ENOMEM; }

    /* steps 1-2: local sorts and regular samples */
    uint64_t ns = 0;
    for (uint32_t b = 0; b < B; b++) {
        uint64_t lo = (uint64_t)b * N / B, hi = (uint64_t)(b + 1) * N / B;
        uint64_t w = hi - lo;
        for (uint64_t x = lo; x < hi; x++) { blk[x].r = R[x]; blk[x].i = (uint32_t)x; }
        qsort(blk + lo, w, sizeof(orc_key), orc_key_cmp);
        for (uint32_t t = 1; t < B; t++) smp[ns++] = blk[lo + (uint64_t)t * w / B];
    }
    /* step 3: sorted samples and pivots */
    qsort(smp, ns, sizeof(orc_key), orc_key_cmp);
    for (uint32_t i = 1; i < B; i++) {
        uint64_t pos = (uint64_t)(i - 1) * B + B / 2 - 1;
        piv[i - 1] = smp[pos];
        if (piv_r) piv_r[i - 1] = smp[pos].r;
        if (piv_i) piv_i[i - 1] = smp[pos].i;
    }
    /* step 4: bucket of every key = pivots strictly below it */
    for (uint32_t x = 0; x < N; x++) {
        orc_key k = { R[x], x };
        uint32_t b = 0;
        for (uint32_t p = 0; p + 1 < B; p++) b += orc_key_lt(piv[p], k);
        bucket[x] = b;
    }
    /* grouped order: bucket by bucket, each bucket in key order */
    for (uint32_t x = 0; x < N; x++) fill[bucket[x] + 1]++;
    offsets[0] = 0;
    for (uint32_t b = 0; b < B; b++) offsets[b + 1] = offsets[b] + fill[b + 1];
    for (uint32_t b = 0; b < B; b++) fill[b] = offsets[b];
    for (uint32_t x = 0; x < N; x++) {
        uint32_t p = fill[bucket[x]]++;
        blk[p].r = R[x]; blk[p].i = x;
    }
    for (uint32_t b = 0; b < B; b++)
        qsort(blk + offsets[b], offsets[b + 1] - offsets[b], sizeof(orc_key), orc_key_cmp);
    for (uint32_t x = 0; x < N; x++) order[x] = blk[x].i;

    free(blk); free(smp); free(piv); free(fill);
    return ORC_OK;
}

/* ---- globalized k-mer rank (Section 3.1.1, Algorithm 2 steps 1-6) ---- */

/* One d(i,j) term (Equations 1-2). */
static double orc_pair_distance(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                                const uint32_t *K, uint32_t i, uint32_t j, double delta)
{
    uint32_t s = orc_shared(ids + off[i], cnt + off[i], off[i + 1] - off[i],
                            ids + off[j], cnt + off[j], off[j + 1] - off[j]);
    uint32_t D = K[i] < K[j] ? K[i] : K[j];
    return orc_distance(orc_fraction(s, D), delta);
}

/* Steps 1-2: processor b holds the contiguous input block
 * [floor(bN/B), floor((b+1)N/B)) of w_b sequences and ranks each of them
 * against its own block only: R_i = (1/w_b) sum_{j in block} d(i,j), j = i
 * included, in increasing j with Neumaier-compensated addition. */
int orc_local_ranks(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                    const uint32_t *K, uint32_t N, uint32_t B, double delta, double *out)
{
    if (B == 0 || B > N) return ORC_EINVAL;
    for (uint32_t b = 0; b < B; b++) {
        uint64_t lo = (uint64_t)b * N / B, hi = (uint64_t)(b + 1) * N / B;
        for (uint64_t i = lo; i < hi; i++) {
            double sum = 0.0, comp = 0.0;
            for (uint64_t j = lo; j < hi; j++) {
                double d = orc_pair_distance(ids, cnt, off, K, (uint32_t)i, (uint32_t)j, delta);
                double t = sum + d;
                if (fabs(sum) >= fabs(d)) comp += (sum - t) + d;
                else comp += (d - t) + sum;
                sum = t;
            }
            out[i] = (sum + comp) / (double)(hi - lo);
        }
    }
    return ORC_OK;
}

/* Steps 3-4: each processor sorts its block by key (local rank, index) and
 * picks k sequences at the evenly spaced 0-based positions
 * floor(t * w_b / (k+1)), t = 1..k (the regular-sampling rule of the split
 * with k in place of B-1; with k = w_b every sequence is picked).  Step 5
 * gathers them: samples[b*k + t-1] = input index, block by block.
 * Requires 1 <= k <= w_b for every block. */
int orc_global_samples(const double *local, uint32_t N, uint32_t B, uint32_t k, uint32_t *samples)
{
    if (B == 0 || B > N || k == 0) return ORC_EINVAL;
    orc_key *blk = (orc_key *)malloc(sizeof(orc_key) * N);
    if (!blk) return ORC_ENOMEM;
    for (uint32_t b = 0; b < B; b++) {
        uint64_t lo = (uint64_t)b * N / B, hi = (uint64_t)(b + 1) * N / B, w = hi - lo;
        if (k > w) { free(blk); return ORC_EINVAL; }
        for (uint64_t x = lo; x < hi; x++) { blk[x].r = local[x]; blk[x].i = (uint32_t)x; }
        qsort(blk + lo, w, sizeof(orc_key), orc_key_cmp);
        for (uint32_t t = 1; t <= k; t++)
            samples[(uint64_t)b * k + t - 1] = blk[lo + (uint64_t)t * w / (k + 1)].i;
    }
    free(blk);
    return ORC_OK;
}

/* Step 6: every sequence re-ranked against the S = k*B gathered samples,
 * R_i = (1/S) sum_{s} d(i, samples[s]) in sample order (a sample is ranked
 * against itself too), Neumaier-compensated; scale[q] = (1/S) sum |d|. */
void orc_global_rank_rows(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                          const uint32_t *K, const uint32_t *samples, uint32_t S,
                          const uint32_t *rows, uint32_t nrows, double delta, double *out,
                          double *scale)
{
    for (uint32_t q = 0; q < nrows; q++) {
        uint32_t i = rows[q];
        double sum = 0.0, comp = 0.0, mag = 0.0;
        for (uint32_t x = 0; x < S; x++) {
            double d = orc_pair_distance(ids, cnt, off, K, i, samples[x], delta);
            double t = sum + d;
            if (fabs(sum) >= fabs(d)) comp += (sum - t) + d;
            else comp += (d - t) + sum;
            sum = t;
            mag += fabs(d);
        }
        out[q] = (sum + comp) / (double)S;
        if (scale) scale[q] = mag / (double)S;
    }
}

/* ---- per-bucket distance matrix and guide tree ---- */

/* Equations 1-2 for the pairs rows[0..nr) x cols[0..nc):
 * out[r*nc + c] = d(rows[r], cols[c]) (F = 1 when both are the same
 * sequence). */
void orc_distance_block(const uint16_t *ids, const uint16_t *cnt, const uint64_t *off,
                        const uint32_t *K, const uint32_t *rows, uint32_t nr, const uint32_t *cols,
                        uint32_t nc, double delta, double *out)
{
    for (uint32_t r = 0; r < nr; r++)
        for (uint32_t c = 0; c < nc; c++)
            out[(uint64_t)r * nc + c] = orc_pair_distance(ids, cnt, off, K, rows[r], cols[c], delta);
}

/* UPGMA (unweighted pair-group method with arithmetic mean, i.e. average
 * linkage) on an n x n dissimilarity matrix d, of which only the upper
 * triangle (r < c) is read.
 *
 * Clusters live in slots: leaf i starts in slot i with id i.  Step t
 * (t = 0 .. n-2) takes, among the active slots a < b, the pair with the
 * smallest D[a][b], ties broken by the smallest a, then the smallest b;
 * the merged cluster gets id n + t and slot a, slot b is retired, and for
 * every other active slot k
 *     D[a,k] = (n_a D[a,k] + n_b D[b,k]) / (n_a + n_b)
 * evaluated as written in IEEE double (two products, one sum, one
 * quotient), with n_a, n_b the cluster sizes and D[x,y] meaning the entry
 * of the upper triangle.  Outputs per step: merges[2t] < merges[2t+1], the
 * two ids merged, and heights[t] = D[a][b] / 2. */
int orc_upgma(const double *d, uint32_t n, int32_t *merges, double *heights)
{
    if (n == 0) return ORC_EINVAL;
    double *D = (double *)malloc(sizeof(double) * (size_t)n * n);
    uint32_t *size = (uint32_t *)malloc(sizeof(uint32_t) * n);
    int32_t *id = (int32_t *)malloc(sizeof(int32_t) * n);
    uint8_t *act = (uint8_t *)malloc(n);
    if (!D || !size || !id || !act) { free(D); free(size); free(id); free(act); return ORC_ENOMEM; }
    memcpy(D, d, sizeof(double) * (size_t)n * n);
    for (uint32_t i = 0; i < n; i++) { size[i] = 1; id[i] = (int32_t)i; act[i] = 1; }
#define UD(x, y) D[(size_t)((x) < (y) ? (x) : (y)) * n + ((x) < (y) ? (y) : (x))]
    for (uint32_t t = 0; t + 1 < n; t++) {
        uint32_t ba = 0, bb = 0;
        int found = 0;
        for (uint32_t a = 0; a < n; a++) {
            if (!act[a]) continue;
            for (uint32_t b = a + 1; b < n; b++) {
                if (!act[b]) continue;
                if (!found || D[(size_t)a * n + b] < D[(size_t)ba * n + bb]) {
                    ba = a; bb = b; found = 1;
                }
            }
        }
        const double h = D[(size_t)ba * n + bb];
        const int32_t x = id[ba], y = id[bb];
        merges[2 * t] = x < y ? x : y;
        merges[2 * t + 1] = x < y ? y : x;
        heights[t] = h / 2.0;
        const double na = (double)size[ba], nb = (double)size[bb];
        for (uint32_t k = 0; k < n; k++) {
            if (!act[k] || k == ba || k == bb) continue;
            const double p = na * UD(ba, k);
            const double q = nb * UD(bb, k);
            const double sum = p + q;
            UD(ba, k) = sum / (na + nb);
        }
        act[bb] = 0;
        size[ba] += size[bb];
        id[ba] = (int32_t)(n + t);
    }
#undef UD
    free(D); free(size); free(id); free(act);
    return ORC_OK;
}

/* ---- profiles and the profile sum of pairs score (Section 3.1.3, Equation 4) ---- */

/* The 20 amino acids of a profile column, in the order of their one-letter
 * codes ACDEFGHIKLMNPQRSTVWY; -1 for anything else. */
static int orc_aa_index(uint8_t ch)
{
    static const char order[] = "ACDEFGHIKLMNPQRSTVWY";
    for (int a = 0; a < 20; a++)
        if (order[a] == ch) return a;
    return -1;
}

/* Profile of an alignment of m rows of L columns (aln row-major): f[x*20+a]
 * = (rows holding amino acid a in column x) / m; the gap characters '-' and
 * '.' count toward no amino acid (the column's gap frequency is 1 minus the
 * sum).  Any other byte returns ORC_EBADRESIDUE with its position in *bad. */
int orc_profile(const uint8_t *aln, uint32_t m, uint32_t L, double *f, uint64_t *bad)
{
    if (m == 0) return ORC_EINVAL;
    for (uint64_t q = 0; q < (uint64_t)L * 20; q++) f[q] = 0.0;
    for (uint32_t r = 0; r < m; r++) {
        for (uint32_t x = 0; x < L; x++) {
            const uint8_t ch = aln[(uint64_t)r * L + x];
            if (ch == '-' || ch == '.') continue;
            const int a = orc_aa_index(ch);
            if (a < 0) { if (bad) *bad = (uint64_t)r * L + x; return ORC_EBADRESIDUE; }
            f[(uint64_t)x * 20 + a] += 1.0;
        }
    }
    for (uint64_t q = 0; q < (uint64_t)L * 20; q++) f[q] /= (double)m;
    return ORC_OK;
}

/* Equation 4 for every column pair: S[x*Ly + y] = sum_i sum_j fx[x][i]
 * fy[y][j] M[i][j], the double sum taken as written (i outer, j inner). */
void orc_psp(const double *fx, uint32_t Lx, const double *fy, uint32_t Ly, const double *M, double *S)
{
    for (uint32_t x = 0; x < Lx; x++)
        for (uint32_t y = 0; y < Ly; y++) {
            double sum = 0.0;
            for (int i = 0; i < 20; i++)
                for (int j = 0; j < 20; j++)
                    sum += fx[(uint64_t)x * 20 + i] * fy[(uint64_t)y * 20 + j] * M[i * 20 + j];
            S[(uint64_t)x * Ly + y] = sum;
        }
}

/* The log-odds term of Equation 4 from a joint distribution P of aligned
 * amino-acid pairs: M[i][j] = log(P[i][j] / (p_i p_j)) with the background
 * probabilities p_i = sum_j P[i][j] (P summing to 1, every entry > 0). */
int orc_psp_matrix(const double *P, double *M)
{
    double p[20];
    for (int i = 0; i < 20; i++) {
        p[i] = 0.0;
        for (int j = 0; j < 20; j++) {
            if (!(P[i * 20 + j] > 0.0)) return ORC_EINVAL;
            p[i] += P[i * 20 + j];
        }
    }
    for (int i = 0; i < 20; i++)
        for (int j = 0; j < 20; j++) M[i * 20 + j] = log(P[i * 20 + j] / (p[i] * p[j]));
    return ORC_OK;
}

