/*
 * kd.h - C ABI of libkmerdecomp, the MI355X (gfx950) implementation of the
 * data-parallel front end of Sample-Align-D (Saeed & Khokhar, "A Domain
 * Decomposition Strategy for Alignment of Multiple Biological Sequences on
 * Multiprocessor Platforms"): per-sequence k-mer counting, all-pairs k-mer
 * similarity, the k-mer rank of every sequence, and the rank-ordered
 * regular-sampling split of the set into B buckets.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every array argument is a DEVICE pointer (HBM of the context's GPU),
 *    caller-owned unless stated otherwise.  Work is enqueued on the context's
 *    stream and reads/writes happen in that stream's order; a call returns
 *    after enqueueing unless its description says it synchronizes.
 *  - Status codes are negative on error.  No C++ exception crosses this ABI.
 *    On error nothing is returned through `out` parameters; output arrays
 *    are left unspecified only where the description says so.
 *  - One context per host thread.  Contexts are not internally synchronized
 *    (the server object below is).  A counted set belongs to the context
 *    that counted it: every call taking a set and a context requires that
 *    context (KD_EINVAL otherwise).
 *  - Alphabet and word length: k = 6 over the Dayhoff-6 grouping of the 20
 *    standard amino acids {AGPST}{C}{DENQ}{FWY}{HKR}{ILMV}; word w of a
 *    sequence is the base-6 number of the group codes of residues w..w+5,
 *    first residue most significant (0 <= w < 46656).  Upper-case ASCII
 *    only; any other byte is rejected.
 */
#ifndef KD_H
#define KD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t kd_status;

#define KD_OK 0
#define KD_EINVAL (-1)        /* bad argument: NULL, B == 0, B > n, bad offsets, delta <= 0 ... */
#define KD_EBADRESIDUE (-2)   /* a byte outside the 20 standard amino acids */
#define KD_ESHORTSEQ (-3)     /* a sequence with fewer than k = 6 residues */
#define KD_ETOOLONG (-4)      /* a sequence with more than 65535 k-mers */
#define KD_ENOMEM (-5)        /* device allocation failed */
#define KD_EBUSY (-6)         /* server: job does not fit the HBM budget right now */
#define KD_EDEVICE (-7)       /* a HIP runtime error */
#define KD_ECANCELLED (-8)    /* server: job was cancelled */
#define KD_ETOOLARGE (-9)     /* input beyond a call's fixed maximum size */

#define KD_K 6
#define KD_WORDS 46656        /* 6^6 distinct words */
#define KD_MAX_KMERS 65535    /* per sequence: n - k + 1 must not exceed this */

typedef struct kd_ctx kd_ctx;
typedef struct kd_set kd_set;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a
 * hipStream_t; NULL is the device's null stream, the one PyTorch uses by
 * default).  The stream stays caller-owned.  The context owns a device
 * memory pool that is released by kd_ctx_destroy. */
kd_status kd_ctx_create(int device, void *hip_stream, kd_ctx **out);
void kd_ctx_destroy(kd_ctx *ctx);
const char *kd_strerror(kd_status status);
/* Sequence index and residue position of the last KD_EBADRESIDUE /
 * KD_ESHORTSEQ / KD_ETOOLONG reported on this context. */
kd_status kd_last_error_info(const kd_ctx *ctx, uint64_t *seq, uint64_t *pos);
/* Block until all work enqueued on the context's stream has finished. */
kd_status kd_ctx_synchronize(kd_ctx *ctx);
/* The hipStream_t the context enqueues on. */
void *kd_ctx_stream(kd_ctx *ctx);

/* Stage timing.  While enabled, the context records a pair of HIP events on
 * its stream around every stage it enqueues; kd_ctx_stage_time synchronizes
 * the stream and returns the summed elapsed milliseconds and the number of
 * timed launches of one stage since the last reset.  kd_ctx_enable_timing
 * takes 0 (off), 1 (every stage) or KD_TIME_MASK | (bit per stage) to time
 * only some stages (each timed stage costs two event records). */
#define KD_STAGE_COUNT 0      /* kmer_count: counting kernels */
#define KD_STAGE_LAYOUT 1     /* kmer_count: sort by distinct words, layout */
#define KD_STAGE_PAIRS 2      /* kmer_rank: the all-pairs kernel */
#define KD_STAGE_FINALIZE 3   /* kmer_rank: accumulator clear + finalize */
#define KD_STAGE_PARTITION 4  /* sample_partition */
#define KD_STAGE_SIMILARITY 5 /* kmer_similarity */
#define KD_STAGE_GLOBAL 6     /* kmer_rank_global: every sequence against the samples
                                 (its sample choice is timed as partition, the samples'
                                 layout as count + layout, its finalize as finalize) */
#define KD_STAGE_GATHER 7     /* kd_gather_sequences */
#define KD_STAGE_DIST 8       /* kmer_distance_matrices */
#define KD_STAGE_TREE 9       /* upgma_trees */
#define KD_STAGE_PSP 10       /* psp_profile, psp_scores */
#define KD_NSTAGES 11
#define KD_TIME_MASK 0x10000  /* enable argument: bits 0..10 select stages */
kd_status kd_ctx_enable_timing(kd_ctx *ctx, int enable);
kd_status kd_ctx_stage_time(kd_ctx *ctx, int stage, double *ms, uint64_t *launches);
kd_status kd_ctx_reset_timing(kd_ctx *ctx);

/* ------------------------------------------------------------- kmer_count */

/* Count vectors c^X of every sequence of the set (paper, Section 3, "k-mer
 * Rank": the vector of occurrence counts of each of the epsilon = c^k words).
 *
 *   residues    device u8[n_residues]: the sequences back to back (ASCII)
 *   offsets     device u64[n_seqs+1]: sequence i is residues[offsets[i] ..
 *               offsets[i+1]); offsets[0] = 0, offsets[n_seqs] = n_residues
 *   n_seqs      number of sequences N (0 gives an empty set)
 *   out         receives a library-owned, device-resident kd_set holding the
 *               count vectors in the layout the similarity and rank calls
 *               consume; free it with kd_set_destroy before the context.
 *
 * Synchronizes the stream once (to report input errors and size the set).
 * Errors: KD_EBADRESIDUE / KD_ESHORTSEQ / KD_ETOOLONG for the lowest-indexed
 * offending sequence (kd_last_error_info gives it and the residue position),
 * KD_EINVAL for inconsistent offsets.  Inputs are only read; they may be
 * reused as soon as the call returns. */
kd_status kmer_count(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                     uint32_t n_seqs, uint64_t n_residues, kd_set **out);

uint32_t kd_set_size(const kd_set *set);          /* N */
uint64_t kd_set_entries(const kd_set *set);       /* sum over sequences of distinct words */
/* Export the count vectors as sorted nonzero entries: sequence i owns
 * ids/counts[off[i] .. off[i+1]) in increasing word order.  ids and counts
 * are device u16[kd_set_entries], off is device u64[N+1]. */
kd_status kd_set_export_lists(kd_ctx *ctx, const kd_set *set, uint16_t *ids, uint16_t *counts,
                              uint64_t *off);
/* Export dense count vectors of sequences first..first+count-1 as a device
 * u16[count x 46656] row-major array. */
kd_status kd_set_export_dense(kd_ctx *ctx, const kd_set *set, uint32_t first, uint32_t count,
                              uint16_t *out);
void kd_set_destroy(kd_set *set);

/* -------------------------------------------------------- kmer_similarity */

/* Common k-mer counts of a block of pairs (Section 3: C_i = min(c^X_i, c^Y_i)
 * summed over all words, the numerator of Equation 1) and, optionally, the
 * Equation 1 denominators min(n, m) - k + 1.
 *
 *   rows r0 .. r0+nr-1 and columns c0 .. c0+nc-1 (sequence indices of `set`)
 *   shared  device u16[nr x nc], row-major: shared[r*nc + c] for the pair
 *           (r0 + r, c0 + c)
 *   denom   device u16[nr x nc] or NULL
 * Errors: KD_EINVAL when the block leaves [0, N). */
kd_status kmer_similarity(kd_ctx *ctx, const kd_set *set, uint32_t r0, uint32_t nr, uint32_t c0,
                          uint32_t nc, uint16_t *shared, uint16_t *denom);

/* -------------------------------------------------------------- kmer_rank */

/* k-mer rank of every sequence (Equation 3): R_i = (1/N) sum_{j=1..N} d(i,j),
 * the sum running over all N sequences including i itself, with
 * d = -ln(delta + F) (Equation 2, natural logarithm) and F the fraction of
 * Equation 1.
 *
 *   delta  the paper's small positive constant (finite, > 0)
 *   ranks  device f64[N], indexed like the input sequences
 * The pairwise sum is accumulated exactly (fixed point), so the result does
 * not depend on scheduling, tiling or what else runs on the device.
 * Errors: KD_EINVAL for delta <= 0 or not finite. */
kd_status kmer_rank(kd_ctx *ctx, const kd_set *set, double delta, double *ranks);

/* Autotuner for the rank kernel's work-list shape.  The all-pairs work of a
 * counted object is cut into about T = t x (compute units) tasks of equal
 * estimated cost (runs of row blocks against strips of 2,048 sequences),
 * which one persistent workgroup per compute unit takes from per-XCD
 * queues; more tasks balance better (and, in a batch, let more compute
 * units of an XCD share one set's column lists in L2), fewer flush fewer
 * column sums to the accumulators.  Without tuning t = 32.  Times
 * kmer_rank on `set` for each of the
 * KD_TUNE_CANDIDATES values t = {8, 16, 32, 64, 128} (one warm-up and three
 * timed runs each; the stream is synchronized), checks that all shapes give
 * bit-identical ranks (KD_EDEVICE otherwise), gives the set the smallest t
 * whose time is within 1% of the fastest (shapes that time alike are told
 * apart by noise; the smaller flushes fewer sums) and remembers t in the
 * context for later counted objects of the same size class (power-of-two
 * bucket of the sequence count, single sets and batches apart).
 *   best    receives the chosen t (may be NULL)
 *   ms_out  NULL or double[KD_TUNE_CANDIDATES]: mean milliseconds per shape */
#define KD_TUNE_CANDIDATES 5
kd_status kd_autotune(kd_ctx *ctx, kd_set *set, double delta, uint32_t *best, double *ms_out);
/* Set t (rank tasks per compute unit, 1..4096) by hand for the size
 * class of (nsets, n); it applies to objects counted afterwards. */
kd_status kd_ctx_set_tasks_per_cu(kd_ctx *ctx, uint32_t nsets, uint32_t n, uint32_t tasks);

/* -------------------------------------------------------- sample_partition */

/* Regular-sampling split of n ranked sequences into B buckets (Section
 * 3.1.2; Algorithm 2 steps 3 and 8-11), with B playing the paper's p:
 *   1. virtual processor b holds input indices [floor(bn/B), floor((b+1)n/B))
 *      and orders them by key (rank, index);
 *   2. it contributes the keys at 0-based positions floor(t w_b / B),
 *      t = 1..B-1, of its ordered block (w_b keys) as regular samples;
 *   3. the B(B-1) samples are ordered and the ones at 0-based positions
 *      (i-1)B + floor(B/2) - 1, i = 1..B-1, become the B-1 pivots;
 *   4. a key goes to the bucket numbered by how many pivots lie strictly
 *      below it, i.e. bucket b holds keys in (pivot_{b-1}, pivot_b].
 * Keys compare by rank, then by index, so all keys are distinct.  With
 * n >= B*B no bucket exceeds 2*ceil(n/B) sequences (Section 3.2).
 *
 *   ranks       device f64[n] (not NaN)
 *   bucket      device u32[n]: bucket of sequence i
 *   order       device u32[n]: sequence indices bucket by bucket, each
 *               bucket in key order (equivalently: all keys in order)
 *   offsets     device u32[B+1]: bucket b is order[offsets[b] .. offsets[b+1])
 *   pivot_rank  device f64[B-1] or NULL; pivot_idx device u32[B-1] or NULL
 * Errors: KD_EINVAL for n == 0, B == 0, B > n or B > 1024. */
kd_status sample_partition(kd_ctx *ctx, const double *ranks, uint32_t n, uint32_t B,
                           uint32_t *bucket, uint32_t *order, uint32_t *offsets,
                           double *pivot_rank, uint32_t *pivot_idx);

/* sample_partition for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, outputs (bit for bit) and errors as
 * sample_partition, plus KD_ETOOLARGE for n > KD_NOALLOC_MAX_KEYS.
 *  - Its working memory is one fixed array of KD_NOALLOC_SCRATCH_BYTES in the
 *    library's device code: each GPU the library runs on holds its own copy
 *    from its first kd_ctx_create until the process ends.  The call makes no
 *    allocation (no hipMalloc, no pool, no pinned staging) and records no
 *    stage timing.
 *  - Nothing in the array has to start at zero: every kernel of the split
 *    writes what it later reads, so a call never depends on what an earlier
 *    call left there.
 *  - Every call on one GPU works in that GPU's one array: calls that overlap
 *    on one GPU (two streams, two contexts, two host threads) race and give
 *    undefined results.  Serialize them, e.g. on one stream. */
#define KD_NOALLOC_MAX_KEYS 1048576u
#define KD_NOALLOC_SCRATCH_BYTES (64ull << 20)
kd_status sample_partition_noalloc(kd_ctx *ctx, const double *ranks, uint32_t n, uint32_t B,
                                   uint32_t *bucket, uint32_t *order, uint32_t *offsets,
                                   double *pivot_rank, uint32_t *pivot_idx);

/* ---------------------------------------------------------------- batches */

/* Many independent sequence sets handled together: every kernel of the
 * count, rank and split runs once over all of them, and each set's result
 * is bit-for-bit what the single-set calls above give for that set alone
 * (the rank accumulation is exact and every set keeps its own tiling).
 *
 * Set s is the sequences set_first[s] .. set_first[s+1]-1 of one input
 * (residues / offsets laid out as for kmer_count, over all sets).
 * set_first is HOST u32[nsets+1] with set_first[0] = 0 and non-decreasing
 * entries; set_B is HOST u32[nsets] (each 1 <= B <= set size, <= 1024). */

/* Count every set; the returned kd_set holds all of them.  kmer_rank on it
 * writes each set's ranks (normalized by that set's size) at the sequences'
 * batch-wide indices; kd_set_export_* cover all sequences; kmer_similarity
 * rejects a set holding more than one set (KD_EINVAL).  Errors as
 * kmer_count, plus KD_EINVAL for a malformed set_first. */
kd_status kmer_count_batch(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                           uint64_t n_residues, uint32_t nsets, const uint32_t *set_first,
                           kd_set **out);
uint32_t kd_set_count(const kd_set *set); /* number of sets it holds */
/* The bounds of its sets: first receives kd_set_count + 1 host u32 values
 * (set s = sequences first[s] .. first[s+1]-1).  Errors: KD_EINVAL for
 * NULL. */
kd_status kd_set_first(const kd_set *set, uint32_t *first);

/* sample_partition of every set, one workgroup per set.
 *   ranks, bucket, order  device f64/u32/u32[set_first[nsets]]; set s uses
 *                         entries set_first[s] .. and its bucket / order
 *                         values are local to the set (0 .. n_s - 1)
 *   offsets               device u32[sum_s (B_s + 1)], set after set
 *   pivot_rank/pivot_idx  device [sum_s (B_s - 1)] or NULL, set after set
 * Errors: KD_EINVAL for a malformed set_first or an invalid B_s. */
kd_status sample_partition_batch(kd_ctx *ctx, const double *ranks, uint32_t nsets,
                                 const uint32_t *set_first, const uint32_t *set_B,
                                 uint32_t *bucket, uint32_t *order, uint32_t *offsets,
                                 double *pivot_rank, uint32_t *pivot_idx);

/* kmer_count_batch + kmer_rank + sample_partition_batch in one call (the
 * counted layout is released on return, in stream order).  Outputs as
 * described for sample_partition_batch; ranks is device f64[set_first[nsets]]. */
kd_status kd_batch_run(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                       uint64_t n_residues, uint32_t nsets, const uint32_t *set_first,
                       const uint32_t *set_B, double delta, double *ranks, uint32_t *bucket,
                       uint32_t *order, uint32_t *offsets_out);

/* A batch set up once and replayed as one HIP graph (the batching pattern
 * of the workloads: all sets in one pass, launched without host work).
 * kd_batch_plan_create takes kd_batch_run's arguments, copies the inputs
 * into device memory of its own, runs the batch once (outputs written; the
 * count's sizing synchronization happens here) while recording each of its
 * kernel launches, and captures them into a graph: counting, layout, the
 * rank launch over every set's work, finalize and the split of every set.
 * kd_batch_plan_launch enqueues the graph on the context's stream: it
 * recomputes the batch from the plan's copy of the inputs and writes the
 * outputs again (bit-identical), with no host synchronization and no
 * allocation.  The plan holds all device memory of the batch until
 * kd_batch_plan_destroy (which synchronizes the stream).  A plan belongs to
 * its context and must be destroyed before it; the output buffers must stay
 * valid while the plan can be launched.  Errors: those of kd_batch_run;
 * KD_EDEVICE if the graph cannot be captured. */
typedef struct kd_batch_plan kd_batch_plan;
kd_status kd_batch_plan_create(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                               uint64_t n_residues, uint32_t nsets, const uint32_t *set_first,
                               const uint32_t *set_B, double delta, double *ranks, uint32_t *bucket,
                               uint32_t *order, uint32_t *offsets_out, kd_batch_plan **out);
kd_status kd_batch_plan_launch(kd_batch_plan *plan);
uint32_t kd_batch_plan_launches(const kd_batch_plan *plan); /* nodes (kernels) of the graph */
void kd_batch_plan_destroy(kd_batch_plan *plan);

/* Algorithm 2 step 1 on one device: the n sequences split into the B
 * contiguous blocks [floor(bn/B), floor((b+1)n/B)) the paper's processors
 * start from, each counted as its own set (kmer_count_batch with those
 * bounds).  kmer_rank on the result gives the local ranks of step 2.
 * Inputs as for kmer_count.  Errors: those of kmer_count_batch; KD_EINVAL
 * for B == 0 or B > n. */
kd_status kmer_count_blocks(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                            uint32_t n_seqs, uint64_t n_residues, uint32_t B, kd_set **out);

/* ------------------------------------------------------- globalized rank */

/* Globalized k-mer rank (Section 3.1.1 "Globalised k-mer Rank"; Algorithm 2
 * steps 3-6), the rank a processor can form without the other processors'
 * sequences.  `blocks` is a counted batch whose sets are the processors'
 * blocks (kmer_count_batch; a single counted set is one block), and
 * local_ranks is kmer_rank(blocks): each sequence ranked against its own
 * block only (steps 1-2).  Then:
 *   3-4. each block is ordered by key (local rank, index) and the sequences
 *        at 0-based positions floor(t w_b / (k+1)), t = 1..k, of its w_b
 *        ordered sequences become its k samples (the split's regular
 *        sampling rule with k in place of B-1);
 *   5.   the k * nsets samples are gathered, block after block;
 *   6.   every sequence is ranked against them:
 *          R_i = (1 / S) sum_{s=1..S} d(i, sample_s),  S = k * nsets,
 *        with d from Equations 1-2 (a sample meets itself as one of the S).
 * The sum is accumulated exactly like kmer_rank's.  Feeding the result to
 * sample_partition(ranks, N, B) with B = nsets finishes Algorithm 2 (steps
 * 7-11).
 *
 *   local_ranks  device f64[N] (not NaN), indexed like the input sequences
 *   k            samples per block, 1 <= k <= the smallest block's size
 *   ranks        device f64[N]: the globalized ranks, indexed like the input
 *   samples      device u32[k * nsets] or NULL: input indices of the samples
 * Device memory: beside small arrays, a temporary of 4 bytes per residue of
 * `blocks`; the stream is synchronized once.
 * Errors: KD_EINVAL for a NULL argument, k out of range, delta <= 0 or not
 * finite, or `blocks` counted on another context. */
kd_status kmer_rank_global(kd_ctx *ctx, const kd_set *blocks, const double *local_ranks,
                           uint32_t k, double delta, double *ranks, uint32_t *samples);

/* ------------------------------------------------------------ decompose */

/* The decomposition front end of Algorithm 2 on one device, in one call:
 * every sequence ranked, then split into B buckets by regular sampling
 * (sample_partition).  The rank is either
 *   KD_RANK_CENTRALIZED  Equation 3 over all n sequences (kmer_rank), or
 *   KD_RANK_GLOBALIZED   the globalized rank of Section 3.1.1: the B blocks
 *                        [floor(bn/B), floor((b+1)n/B)) counted as a batch,
 *                        ranked locally, k = max(1, B-1) samples per block
 *                        (kmer_rank_global).
 * Outputs as for sample_partition, plus ranks (device f64[n]); the results
 * are bit-identical to making those calls one by one.
 * Errors: those of the calls it makes; KD_EINVAL for an unknown mode or a
 * block smaller than k. */
#define KD_RANK_CENTRALIZED 0
#define KD_RANK_GLOBALIZED 1
kd_status kd_decompose(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                       uint32_t n_seqs, uint64_t n_residues, uint32_t B, int mode, double delta,
                       double *ranks, uint32_t *bucket, uint32_t *order, uint32_t *bucket_offsets);

/* ------------------------------------------------- buckets and guide trees */

/* Redistribution on one device (Section 3.1.2: bucket i's sequences go to
 * processor i; Algorithm 2 step 11): sequences order[0..n) of `residues`
 * (input indices, e.g. sample_partition's order) written back to back.
 *   residues, offsets  device u8[n_residues], u64[n_seqs+1] as for kmer_count
 *   out_residues       device u8[out_capacity]
 *   out_offsets        device u64[n+1]: sequence x of the output is
 *                      out_residues[out_offsets[x] .. out_offsets[x+1])
 * The stream is synchronized once (to check the size before copying).
 * Errors: KD_EINVAL for a NULL argument, an entry of order >= n_seqs, a
 * gathered sequence whose offsets decrease or pass n_residues, or a total
 * length above out_capacity (no residue is copied then). */
kd_status kd_gather_sequences(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                              uint32_t n_seqs, uint64_t n_residues, const uint32_t *order,
                              uint32_t n, uint8_t *out_residues, uint64_t out_capacity,
                              uint64_t *out_offsets);

/* The k-mer distance matrix of every set of a counted object: Equations
 * 1-2 for every ordered pair of sequences of the set, the pairwise
 * similarity matrix that a bucket's local alignment starts from (the
 * generic scheme of Section 2, run per bucket in Section 3.1.3).
 *   dist  device f64[sum_s n_s^2]: set s's n_s x n_s matrix, row-major in
 *         the set's input order, starts after the matrices of sets 0..s-1;
 *         the diagonal holds -ln(1 + delta) (F = 1)
 * Errors: KD_EINVAL for delta <= 0 or not finite, a NULL argument, or a set
 * counted on another context. */
kd_status kmer_distance_matrices(kd_ctx *ctx, const kd_set *set, double delta, double *dist);

/* UPGMA (average linkage) guide tree of each of nsets dissimilarity
 * matrices laid out as kmer_distance_matrices writes them (set s has
 * n_s = set_first[s+1] - set_first[s] members; only the upper triangle is
 * read; dist is not modified).  Leaf i of a set is its i-th member; step t
 * merges the two clusters whose slots a < b hold the smallest D[a][b]
 * (ties: smallest a, then smallest b), gives the result id n_s + t and slot
 * a, and sets D[a][k] = (n_a D[a][k] + n_b D[b][k]) / (n_a + n_b) for the
 * other clusters k (rounded after each product, the sum and the quotient).
 *   set_first  host u32[nsets+1], set_first[0] = 0, every set non-empty
 *   merges     device i32[2 * (set_first[nsets] - nsets)]: set s's n_s - 1
 *              steps start at 2 (set_first[s] - s), each the two merged
 *              ids, smaller first
 *   heights    device f64[set_first[nsets] - nsets]: D[a][b] / 2 per step
 * Device memory: a working copy of dist.  The stream is synchronized once.
 * Errors: KD_EINVAL for a NULL argument, a malformed set_first, a set of
 * more than 4096 members, or a matrix whose remaining entries cannot be
 * ordered (NaN). */
kd_status upgma_trees(kd_ctx *ctx, uint32_t nsets, const uint32_t *set_first, const double *dist,
                      int32_t *merges, double *heights);

/* ------------------------------------------------- profiles and PSP scores */

/* Profile of an alignment (Section 3.1.3): for each of its L columns the
 * frequencies of the 20 amino acids, in the order of their one-letter
 * codes ACDEFGHIKLMNPQRSTVWY, over its m rows; '-' and '.' are gaps and
 * count toward no amino acid.
 *   aln  device u8[m x L], row-major (row r = one aligned sequence)
 *   f    device f64[L x 20]: f[x*20 + a] = (rows with amino acid a in
 *        column x) / m
 * Errors: KD_EINVAL for a NULL argument or m == 0; KD_EBADRESIDUE for any
 * other byte (kd_last_error_info: seq = row, pos = column of the first
 * one in row-major order).  The stream is synchronized once. */
kd_status psp_profile(kd_ctx *ctx, const uint8_t *aln, uint32_t m, uint32_t L, double *f);

/* One profile pair for psp_scores (device pointers). */
typedef struct kd_psp_pair {
  const double *fx;  /* f64[lx x 20], profile X */
  uint32_t lx;
  uint32_t ly;
  const double *fy;  /* f64[ly x 20], profile Y */
  double *scores;    /* f64[lx x ly], row-major: scores[x*ly + y] */
} kd_psp_pair;

/* Profile sum of pairs scores (Equation 4) for every column pair of each
 * profile pair: scores[x][y] = sum_i sum_j fx[x][i] fy[y][j] M[i][j], with
 * M[i][j] = log(p_ij / (p_i p_j)) from the caller's substitution model
 * (the paper names PAM 200 and VTML 240; none ships with this library).
 * FP64 throughout (matrix cores).
 *   M      device f64[20 x 20], row-major, amino acids in profile order
 *   pairs  host array of npairs descriptors (pairs with lx or ly 0 are
 *          skipped)
 * Device memory: a temporary of 160 bytes per row of the fx profiles.
 * Errors: KD_EINVAL for a NULL argument, or more than 2^31 tiles of
 * 64 x 512 scores in one call. */
kd_status psp_scores(kd_ctx *ctx, const double *M, uint32_t npairs, const kd_psp_pair *pairs);

/* ------------------------------------------------------------ calibration */

/* Rate of random 16-bit LDS reads, the elementary operation of the rank
 * kernels' mask lookups (measurement support: computes nothing of the
 * method).  Launches `workgroups` workgroups of 1024 threads; every lane
 * makes steps x 32 reads at pseudo-random indices of a 32,768-entry LDS
 * table, `batch` (2, 8 or 32) of them issued together before their values
 * are used.  Synchronizes the stream; returns the kernel's time from HIP
 * events on the context's stream and the number of 64-lane read
 * instructions executed.  Device memory: 4 bytes per thread (freed on
 * return).  Errors: KD_EINVAL for another batch, 0 workgroups or steps,
 * or NULL outputs. */
kd_status kd_calibrate_lds(kd_ctx *ctx, uint32_t workgroups, uint32_t steps, uint32_t batch,
                           double *ms, uint64_t *wave_reads);

/* ----------------------------------------------------------------- server */

/* A request server for many independent jobs (each job = one sequence set
 * to count, rank and split).  A worker thread serves them on `device`: a
 * job is admitted once the device memory it will need fits the budget next
 * to the other admitted jobs and the input mirrors; admitted jobs (of one
 * delta, within the batch limits) are taken together as one batch through
 * kd_batch_run's path, in two stages on two streams of the default
 * priority: (A) gather, count and lay out every set; (B) rank, split and
 * copy the results back.  While a batch is in stage B, the jobs admitted
 * meanwhile start stage A as the next batch, so their counting overlaps
 * the running batch's rank on the device.  Each job's results are
 * bit-for-bit those of running it alone.  All calls are internally
 * synchronized and may come from any thread. */
typedef struct kd_server kd_server;

typedef struct kd_server_opts {
  uint64_t hbm_budget;     /* bytes the admitted jobs may reserve; a job is charged
                              KD_JOB_BYTES(n_residues, n_seqs), an estimate of its
                              peak device memory inside a batch */
  uint32_t max_batch_jobs; /* jobs per batch; 0 = no limit, 1 = one job at a time */
  uint32_t max_batch_seqs; /* sequences per batch; 0 = no limit */
  uint64_t host_arena_bytes; /* pinned host memory for the jobs' input copies, set up at
                                creation (64 MB chunks, kept and reused; more are pinned
                                as jobs need them; a job no chunk can hold keeps a
                                pageable copy).  A chunk gets a device mirror of the same
                                size while the mirrors stay within half of hbm_budget;
                                the mirrors' bytes count against the budget (admission
                                leaves room for them).  A job's residues reach its
                                chunk's mirror at submit, on a copy stream of the
                                server's, while earlier batches run; a job in a chunk
                                without a mirror is sent from the host copy by its
                                batch.  When nonzero, the batch buffers (pinned
                                offsets and results, device input and output) are also
                                set up at creation, for a batch of that many residues in
                                max_batch_seqs sequences (0: a mean length of 128); they
                                grow when a batch needs more */
  uint32_t no_mirror;        /* 1: no device mirrors (no device memory beyond the batch
                                buffers); each batch sends its jobs' residues from
                                their host copies */
  uint32_t timeline;         /* 1: record HIP events around each batch's two stages
                                (kd_server_timeline) */
} kd_server_opts;

#define KD_JOB_BYTES(n_residues, n_seqs) (8ull * (n_residues) + 256ull * (n_seqs) + 65536ull)

typedef struct kd_job {
  const uint8_t *residues;   /* HOST u8[n_residues]; copied by kd_server_submit */
  const uint64_t *offsets;   /* HOST u64[n_seqs+1] as for kmer_count; copied */
  uint32_t n_seqs;
  uint64_t n_residues;
  uint32_t B;                /* buckets: 1 <= B <= n_seqs, B <= 1024 */
  double delta;              /* Equation 2's constant (finite, > 0) */
  double *ranks;             /* HOST f64[n_seqs] or NULL: written before completion */
  uint32_t *bucket;          /* HOST u32[n_seqs] or NULL */
  uint32_t *order;           /* HOST u32[n_seqs] or NULL */
  uint32_t *bucket_offsets;  /* HOST u32[B+1] or NULL */
} kd_job;

typedef struct kd_done {
  uint64_t ticket;
  kd_status status;          /* KD_OK, the job's input error (KD_EBADRESIDUE ...),
                                KD_ECANCELLED or KD_EDEVICE */
  uint32_t batch_jobs;       /* jobs in the batch that served it */
  uint64_t t_submit_ns;      /* CLOCK_MONOTONIC times: submit, batch start, results written */
  uint64_t t_start_ns;
  uint64_t t_done_ns;
} kd_done;

/* Errors: KD_EINVAL for a bad device or NULL arguments, KD_EDEVICE. */
kd_status kd_server_create(int device, const kd_server_opts *opts, kd_server **out);
/* Queue a job; its inputs are copied before this returns (and its residues
 * sent on to the device), its output buffers must stay valid until its
 * kd_done has been polled.  Sets the server's device current for the call
 * and restores the caller's.  Errors:
 * KD_EINVAL (bad offsets, B or delta; detected here), KD_EBUSY (the job
 * alone exceeds the budget). */
kd_status kd_server_submit(kd_server *srv, const kd_job *job, uint64_t *ticket);
/* Move up to `max` completion records into out[0 .. *n); waits up to
 * wait_ns nanoseconds (0: do not wait) when none is ready. */
kd_status kd_server_poll(kd_server *srv, kd_done *out, uint32_t max, uint32_t *n, int64_t wait_ns);
/* Cancel a job that has not started (its record reports KD_ECANCELLED);
 * KD_EBUSY if it is running, KD_EINVAL if the ticket is unknown or done. */
kd_status kd_server_cancel(kd_server *srv, uint64_t ticket);
/* Jobs queued, admitted-and-waiting, running; completion records not yet
 * polled; device bytes reserved: the admitted and running jobs' charges
 * plus the input mirrors (never more than hbm_budget). */
kd_status kd_server_status(kd_server *srv, uint32_t *waiting, uint32_t *admitted,
                           uint32_t *running, uint32_t *done, uint64_t *reserved);
/* One batch's stages on the device (kd_server_opts.timeline): milliseconds
 * from a fixed event recorded at creation to the starts and ends of stage A
 * (gather, count, layout; stream A) and stage B (rank, split, results
 * copied back; stream B).  A batch's stage A may overlap the previous
 * batch's stage B. */
typedef struct kd_server_stage {
  double count_start_ms, count_end_ms;
  double rank_start_ms, rank_end_ms;
  uint32_t jobs;       /* jobs in the batch */
  uint32_t reserved0;
} kd_server_stage;
/* Moves up to `max` records of completed batches, oldest first, into
 * out[0 .. *n). */
kd_status kd_server_timeline(kd_server *srv, kd_server_stage *out, uint32_t max, uint32_t *n);
/* Finishes the running batch, drops queued jobs, joins the worker. */
void kd_server_destroy(kd_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* KD_H */
