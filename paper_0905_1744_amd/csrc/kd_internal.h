// Internal declarations of libkmerdecomp: device layout of a counted set,
// constants of the word space, the device memory pool, kernel launchers and
// the small device helpers several kernels share.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kd.h"

namespace kd {

// ---------------------------------------------------------------- constants

constexpr int kK = 6;                 // word length
constexpr int kWords = 46656;         // 6^6
constexpr uint16_t kSentinel = 46656; // padding word: its table entry stays 0
constexpr int kTableWords = 23329;    // u32 words holding 46658 u16 table slots
constexpr int kBitmapWords = 1458;    // 46656 bits
constexpr int kRowsPerBlock = 16;     // rows sharing one LDS presence table
constexpr int kGroup = 64;            // columns per interleaved group (one per lane)
constexpr int kShortMax = 4096;       // words per sequence handled by the one-wave counter
constexpr uint32_t kMaxBuckets = 1024; // sample_partition: B(B-1) samples stay small

// error word written by the counting kernels: (seq << 32) | (code << 28) | pos
enum : uint32_t { kErrNone = 0, kErrInval = 1, kErrBadResidue = 2, kErrShort = 3, kErrLong = 4 };

// ----------------------------------------------------------- device layout

// A counted set in device memory.  Sequences are re-ordered by ascending
// number of distinct words (ties by input index); "sorted position" s refers
// to that order, perm[s] is the input index and inv[i] its inverse.
//
// A counted object can hold several independent sets (a batch).  Set s owns
// the input sequences base .. base+N-1, the same range of sorted positions,
// and its own column groups and row blocks; all its arrays are views into
// batch-wide arrays, and indices stored in them (perm, inv) are local to the
// set, so every kernel sees one set exactly as if it had been counted alone.
struct SetView {
  uint32_t N;
  uint32_t G;                  // column groups: ceil(N / 64)
  uint32_t RB;                 // row blocks: ceil(N / 16)
  uint32_t base;               // input index of the set's first sequence in the batch
  const uint32_t *perm;        // [N] sorted position -> input index (local)
  const uint32_t *inv;         // [N] input index -> sorted position (local)
  const uint32_t *K;           // [N] words per sequence (n - 5), sorted order
  const uint32_t *D;           // [N] distinct words, sorted order
  const double *invK;          // [N] 1 / K, sorted order
  const uint64_t *grp_off;     // [G+1] u16-element offset of each group in gids
  const uint32_t *grp_len;     // [G] padded list length of the group (multiple of 16)
  const uint16_t *gids;        // interleaved distinct words: element t of the
                               // sequence in lane l of group g lives at
                               // grp_off[g] + ((t/8)*64 + l)*8 + t%8
  const uint32_t *hi_off;      // [N+1] entries with count >= 2, sorted order
  const uint16_t *hi_ids;
  const uint16_t *hi_cnt;
  const uint32_t *ghi;         // count>=2 entries per column group, interleaved like
                               // gids (entry t of lane l at ghi_off[g] + 64 t + l),
                               // packed word | count << 16, zero padded
  const uint64_t *ghi_off;     // [G+1]
  const uint32_t *ghi_len;     // [G] entries per lane, multiple of 4
  const uint32_t *exc_off;     // [RB+1] per row block: merged count>=2 words
  const uint32_t *exc_n;       // [RB] used entries in the block's range
  const uint16_t *exc_ids;     // [cap] sorted words
  const uint16_t *exc_cnt;     // [cap*16] count of the word in each of the 16 rows
  long long *acc;              // [N] exact rank accumulators (fixed point, fix_bits)
};

// Batch-wide numbering: set s holds sequences seq[s] .. seq[s+1]-1, column
// groups grp[s] .. grp[s+1]-1 and row blocks rb[s] .. rb[s+1]-1.
struct Segs {
  uint32_t nsets;
  const uint32_t *seq;     // device [nsets+1]
  const uint32_t *grp;     // device [nsets+1]
  const uint32_t *rb;      // device [nsets+1]
  const SetView *views;    // device [nsets]
  // set of each sorted position / column group / row block (device; only
  // built when nsets > 1)
  const uint32_t *pos_set, *grp_set, *rb_set;
#ifdef __HIPCC__
  __device__ uint32_t set_of_pos(uint32_t p) const { return nsets == 1 ? 0u : pos_set[p]; }
  __device__ uint32_t set_of_grp(uint32_t x) const { return nsets == 1 ? 0u : grp_set[x]; }
  __device__ uint32_t set_of_rb(uint32_t x) const { return nsets == 1 ? 0u : rb_set[x]; }
#endif
};

struct PairTask {     // one workgroup's work in the rank kernel
  uint32_t set;       // index into the SetView array
  uint32_t rb0, rb1;  // row blocks [rb0, rb1), processed one after another
  uint32_t g0;        // column groups g0 .. g0+15, one per wave
};
constexpr uint32_t kGroupsPerTask = 32;  // two column groups per wave
// Per-XCD queues of a rank work list: queue x is tasks[beg[x] .. beg[x+1]),
// head[x] counts the tasks taken from it (zero before every launch).
constexpr uint32_t kXcdQueues = 8;
struct TaskQueues {
  uint32_t beg[kXcdQueues + 1];
  uint32_t *head;  // device [kXcdQueues]
};
struct CrossTask {    // one workgroup's work in the globalized-rank pass
  uint32_t gx0;       // its column groups are gperm[gx0 .. gx0+gpt-1], gpt = 16 or
                      // 32 (batch-wide numbering, 0xFFFFFFFF = none)
  uint32_t rb0, rb1;  // row blocks [rb0, rb1) of the sample set
};
constexpr uint32_t kTasksPerCu = 32;  // default rank tasks per compute unit (kd_autotune)
constexpr size_t kGidsSlack = 16384;  // sentinel words after the last group (read-ahead)

// ---------------------------------------------------------- host objects

class Pool {  // caching device allocator (one per context)
 public:
  Pool() = default;
  ~Pool();
  void *alloc(size_t bytes);
  void free(void *p);
  size_t live_bytes() const { return live_; }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void *>> free_;
  std::map<void *, size_t> size_;
  size_t live_ = 0;
};

}  // namespace kd

struct kd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;  // caller's stream (nullptr: null stream)
  kd::Pool *pool = nullptr;
  uint64_t err_seq = 0, err_pos = 0;
  int cus = 256;
  void *pinned = nullptr;         // small pinned readback area
  void *readback = nullptr;       // growable pinned readback area (read after a sync)
  size_t readback_cap = 0;
  // tuned rank workgroups per compute unit, by size class (kd_autotune)
  std::map<uint32_t, uint32_t> tpc_pref;
  // pinned upload buffers: host data is staged here and copied on the
  // context's stream; a buffer is reused once its copy's event completed
  struct Staged { void *p; size_t cap; hipEvent_t ev; bool used; };
  std::vector<Staged> staging;
  // stage timing (kd_ctx_enable_timing)
  uint32_t timing = 0;  // bit per stage
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_free;  // recycled timing events
  double stage_ms[KD_NSTAGES] = {0};
  uint64_t stage_n[KD_NSTAGES] = {0};
  // while a batch plan is made: every kernel launch of the batch is also
  // kept here (to be replayed into a HIP graph), and pool blocks that would
  // be released at the end of a call are handed to the plan instead
  std::vector<std::function<hipError_t(hipStream_t)>> *rec = nullptr;
  std::vector<void *> *rec_keep = nullptr;
  hipEvent_t wait_ev = nullptr;  // polled by the count's sizing wait
};

struct kd_set {
  kd_ctx *ctx = nullptr;
  kd::SetView v{};        // batch-wide arrays (N, G, RB are totals); equals views[0] for one set
  uint32_t nsets = 1;
  std::vector<kd::SetView> views;                      // per set (host copy)
  std::vector<uint32_t> seq_first, grp_first, rb_first;  // host copies of the segment bounds
  kd::Segs segs{};                                     // device copies
  kd::SetView *d_view = nullptr;  // device copy of views
  kd::PairTask *tasks = nullptr;  // rank work list of all sets (device)
  uint32_t ntasks = 0;
  std::vector<kd::PairTask> h_tasks;
  kd::TaskQueues queues{};  // per-XCD queues over tasks (head: device, in the set's blocks)
  std::vector<uint32_t> h_grp_len;  // padded list length of every column group (host copy)
  mutable bool acc_clean = true;  // rank accumulators are zero (kmer_rank keeps them so)
  uint64_t entries = 0;   // sum of D
  uint64_t cap = 0;       // sum of K
  uint64_t n_hi = 0;      // entries with count >= 2
  uint64_t n_gids = 0;
  uint64_t n_exc = 0;
  std::vector<void *> blocks;  // pool blocks owned by the set
  // per-input-index lists as produced by counting (kept for export):
  // sequence i at cap_ids/cap_cnt[in_off[i] - 5i ...], Dorig[i] entries
  uint16_t *cap_ids = nullptr, *cap_cnt = nullptr;
  uint32_t *Dorig = nullptr;
  uint64_t *in_off = nullptr;
};

namespace kd {

// ------------------------------------------------------------ launchers

// Per input sequence i, at capacity offset offsets[i] - 5i: distinct words
// (cap_ids) and counts (cap_cnt) in word order, and the entries with count
// >= 2 packed as word | count << 16 (hi_cap); D, K and the number of such
// entries.  Also copies the offsets into in_off (N+1 entries).
hipError_t launch_count(hipStream_t st, const uint8_t *res, const uint64_t *off, uint64_t *in_off,
                        uint32_t N, uint64_t nres, uint64_t cap, uint16_t *cap_ids, uint16_t *cap_cnt,
                        uint32_t *hi_cap, uint32_t *Dorig, uint32_t *Korig, uint32_t *nhi_orig,
                        uint32_t *mid_list, uint32_t *nmid, uint32_t *long_list, uint32_t *nlong,
                        uint32_t *next_chunk, unsigned long long *err, int cus);

// per set s: stable sort of (key u32 < 2^16, value = local index) over the
// set's range of keys; writes perm (local indices) over the same range.
// host_first = the set bounds on the host; scratch holds
// sort_scratch_bytes(largest set) bytes.
hipError_t launch_sort_u32_index(hipStream_t st, const uint32_t *keys, const Segs &sg,
                                 const uint32_t *host_first, uint32_t *perm, void *scratch);
size_t sort_scratch_bytes(uint32_t max_n);

struct LayoutMeta {  // totals written by layout_meta, read by the host
  unsigned long long err;
  unsigned long long n_hi;
  unsigned long long n_gids;
  unsigned long long n_exc;
  unsigned long long entries;
  unsigned long long max_len;  // longest padded group list
  unsigned long long n_ghi;    // grouped count>=2 entries incl. padding
};

hipError_t launch_layout_meta(hipStream_t st, const Segs &sg, uint32_t N, uint32_t G,
                              uint32_t RB, const uint32_t *perm,
                              const uint32_t *Dorig, const uint32_t *Korig,
                              const uint32_t *nhi_orig, uint32_t *inv, uint32_t *K, uint32_t *D,
                              double *invK, uint32_t *hcount,
                              uint32_t *hi_off, uint64_t *grp_off, uint32_t *grp_len,
                              uint64_t *ghi_off, uint32_t *ghi_len,
                              uint32_t *exc_off, const unsigned long long *err, LayoutMeta *meta,
                              void *scratch);  // meta must be zeroed beforehand

// scratch bytes launch_layout_meta needs
size_t layout_meta_scratch_bytes(uint32_t N, uint32_t G, uint32_t RB);

hipError_t launch_layout_fill(hipStream_t st, const Segs &sg, const SetView &v,
                              const uint64_t *offsets,
                              const uint16_t *cap_ids, const uint32_t *hi_cap,
                              uint16_t *gids, uint16_t *hi_ids, uint16_t *hi_cnt, uint32_t *ghi,
                              uint32_t max_len);

// merged count>=2 words of row blocks.  rowpos == nullptr: every row block
// of every set (batch-wide numbering); otherwise block b of the first set
// holds the sorted positions rowpos[16b .. 16b+15]
hipError_t launch_exc_build(hipStream_t st, const Segs &sg, uint32_t nblocks,
                            const uint32_t *rowpos, const uint32_t *exc_off, uint32_t *exc_n,
                            uint16_t *exc_ids, uint16_t *exc_cnt);

hipError_t launch_rank_pairs(hipStream_t st, const SetView *d_views, const PairTask *tasks,
                             uint32_t ntasks, const TaskQueues &q, uint32_t workgroups, double delta);
// also clears the queue heads of the rank launch before it
hipError_t launch_rank_finalize(hipStream_t st, const Segs &sg, uint32_t N, double delta,
                                double *ranks, uint32_t *qhead);
// globalized rank: sample rows against every column group of `cols`
hipError_t launch_rank_cross(hipStream_t st, const Segs &cols, const SetView *rows,
                             const CrossTask *tasks, uint32_t ntasks, const uint32_t *gperm,
                             uint32_t gpt, double delta);
hipError_t launch_cross_finalize(hipStream_t st, const Segs &sg, uint32_t N, uint32_t S,
                                 double delta, double *ranks);
// host: the cross pass's work list and column-group permutation from the
// groups' padded list lengths; returns the groups per task (16 or 32)
uint32_t make_cross_tasks(const uint32_t *grp_len, uint32_t Gtot, uint32_t RBs, int cus,
                          std::vector<CrossTask> &out, std::vector<uint32_t> &gperm);
// samples[q*k + t-1] = first[q] + order[first[q] + floor(t w_q / (k+1))]
// (order: each set's local indices in key order); first on the device
hipError_t launch_pick_samples(hipStream_t st, const uint32_t *first, uint32_t nsets, uint32_t k,
                               const uint32_t *order, uint32_t *samples);
// Per-input arrays of a set made of S sequences of a counted parent (input
// indices picks[0..S)), as the counting kernels would have left them:
// Dorig, Korig, count>=2 entries (hi_cap, packed word | count << 16) and
// offsets chosen so that sample s's capacity base offsets[s] - 5s is the
// parent's base for its sequence -- its lists stay in the parent's cap_ids /
// cap_cnt, and hi_cap must be sized like them.
hipError_t launch_gather_samples(hipStream_t st, const Segs &parent, const uint64_t *par_in_off,
                                 const uint32_t *par_Dorig, const uint32_t *picks, uint32_t S,
                                 uint64_t *in_off, uint32_t *Dorig, uint32_t *Korig,
                                 uint32_t *nhi, uint32_t *hi_cap);
// redistribution: out_off = exclusive sums of the lengths of order[0..n)
// (n+1 entries), then (out != nullptr) the bytes; entries of order >=
// n_seqs or with offsets decreasing or past nres set *err, sequences past
// cap are not copied
hipError_t launch_gather(hipStream_t st, const uint8_t *res, const uint64_t *off, uint32_t n_seqs,
                         uint64_t nres, const uint32_t *order, uint32_t n, uint8_t *out, uint64_t cap,
                         uint64_t *out_off, unsigned long long *err);
// Equations 1-2 for every pair of every set, set q's n_q x n_q matrix at
// dist + doff[q] (input order)
constexpr uint32_t kDistLdsRow = 4096;  // larger sets: permutation reads the scratch row in memory
// scratch: each set's matrix in sorted order, rows of dist_ld(n) = n rounded
// up to 16 doubles, set q at soff[q]; dist: input order, set q at doff[q]
hipError_t launch_distances(hipStream_t st, const Segs &sg, uint32_t N, uint32_t max_n, const SetView *d_views,
                            const PairTask *tasks, uint32_t ntasks, const uint64_t *soff, const uint64_t *doff,
                            double delta, double *scratch, double *dist);
constexpr uint32_t kTreeMaxSeqs = 4096;  // largest set upgma_trees accepts
// UPGMA of each set's matrix at work + doff[q] (overwritten), first[] on
// the device (N = first[nsets] members in all, max_n in the largest set);
// rmin/rarg: N entries of scratch; a set with no comparable pair left
// records its index in *err
hipError_t launch_upgma(hipStream_t st, uint32_t nsets, uint32_t N, uint32_t max_n, const uint32_t *first,
                        const uint64_t *doff, double *work, double *rmin, uint32_t *rarg,
                        int32_t *merges, double *heights, unsigned long long *err);
// PSP (Equation 4): profiles of alignments and score matrices of pairs
struct PspWork {  // one pair: the caller's descriptor and its G = fX M scratch
  const double *fx;
  const double *fy;
  double *scores;
  double *g;        // [lx x 20]
  uint32_t lx, ly;
  uint32_t gblk0;   // first 64-row block of the pair in the G kernel's grid
  uint32_t tile0;   // first (64-row x 4-piece) tile of the pair in the score kernel's grid
};
hipError_t launch_psp_profile(hipStream_t st, const uint8_t *aln, uint32_t m, uint32_t L, double *f,
                              unsigned long long *bad);
// host: sets each descriptor's gblk0 / tile0 (its first block in the two
// kernels' compact grids) and returns the totals; false if a grid would be
// too large for one launch
bool psp_plan(std::vector<PspWork> &w, uint64_t &gblks, uint64_t &tiles);
hipError_t launch_psp_scores(hipStream_t st, const PspWork *w, uint32_t npairs, uint32_t gblks,
                             uint32_t tiles, const double *M);
// calibration: steps x 32 random 16-bit LDS reads per lane, `batch` at a time
hipError_t launch_lds_probe(hipStream_t st, uint32_t workgroups, uint32_t steps, uint32_t batch,
                            uint32_t *sink);
hipError_t launch_fill_u64(hipStream_t st, void *p, uint64_t n_words, uint64_t value);
// writes the set ids of sg.pos_set / grp_set / rb_set (nsets > 1)
hipError_t launch_seg_ids(hipStream_t st, const Segs &sg, uint32_t *pos_set, uint32_t *grp_set,
                          uint32_t *rb_set);
struct FillJob {  // n 64-bit words at p set to v
  unsigned long long *p;
  uint64_t n;
  unsigned long long v;
};
struct FillJobs {
  FillJob j[4];
  uint32_t n;
};
hipError_t launch_fills(hipStream_t st, const FillJobs &jobs);  // all jobs in one launch

hipError_t launch_similarity(hipStream_t st, const SetView &v, const uint32_t *rowpos,
                             uint32_t nr, const uint32_t *colpos, uint32_t nc,
                             const uint32_t *exc_off, const uint32_t *exc_n,
                             const uint16_t *exc_ids, const uint16_t *exc_cnt, uint16_t *shared,
                             uint16_t *denom);
hipError_t launch_map_positions(hipStream_t st, const uint32_t *inv, uint32_t first, uint32_t n,
                                uint32_t *pos);
hipError_t launch_exc_offsets(hipStream_t st, const SetView &v, const uint32_t *rowpos,
                              uint32_t nrows, uint32_t *exc_off);

hipError_t launch_export_lists(hipStream_t st, const kd_set *s, uint16_t *ids, uint16_t *counts,
                               uint64_t *off);
hipError_t launch_export_dense(hipStream_t st, const kd_set *s, uint32_t first, uint32_t count,
                               uint16_t *out);

// one regular-sampling split per set of a batch, one workgroup each
struct PartDesc {
  uint64_t scratch_off;  // byte offset of the set's scratch
  uint32_t first;        // first key (ranks, bucket and order are indexed from here)
  uint32_t n, B;
  uint32_t off_base;     // first entry of the set's B+1 offsets
  uint32_t piv_base;     // first entry of the set's B-1 pivots
};
// max_keys: the largest n or B(B-1) of the sets (picks the workgroup size)
hipError_t launch_partition_batch(hipStream_t st, const PartDesc *desc, uint32_t nsets,
                                  uint32_t max_keys, const double *ranks, uint32_t *bucket,
                                  uint32_t *order, uint32_t *offsets, double *pivot_rank,
                                  uint32_t *pivot_idx, void *scratch);

// scratch needed by launch_partition for n keys and B buckets (bytes)
size_t partition_scratch_bytes(uint32_t n, uint32_t B);
hipError_t launch_partition(hipStream_t st, const double *ranks, uint32_t n, uint32_t B,
                            uint32_t *bucket, uint32_t *order, uint32_t *offsets,
                            double *pivot_rank, uint32_t *pivot_idx, void *scratch);

// ------------------------------------------------------- device helpers

#ifdef __HIPCC__

__host__ __device__ constexpr uint8_t dayhoff6(uint32_t ch) {
  switch (ch) {
    case 'A': case 'G': case 'P': case 'S': case 'T': return 0;
    case 'C': return 1;
    case 'D': case 'E': case 'N': case 'Q': return 2;
    case 'F': case 'W': case 'Y': return 3;
    case 'H': case 'K': case 'R': return 4;
    case 'I': case 'L': case 'M': case 'V': return 5;
    default: return 255;
  }
}

// Rank accumulators.  Every tile's FP64 row and column sums are rounded to
// integer multiples of 2^-F and added as 64-bit integers, so a total does
// not depend on the order of its additions (scheduling, tiling, batching).
// F is the largest value with n * dmax * 2^F < 2^62, n the number of terms
// of a rank sum and dmax = max(|ln delta|, ln(1 + delta)) >= |d| for every
// d = -ln(delta + F_xy) with 0 <= F_xy <= 1 (Equation 2), so neither a tile
// sum nor any partial total can overflow.  Every kernel that touches an
// accumulator derives F with this same function.
__host__ __device__ inline int fix_bits(uint32_t n, double delta) {
  const double dmax = fmax(fabs(log(delta)), log1p(delta));
  return 61 - ilogb((double)n * dmax);
}

__host__ __device__ inline long long fix_q(double v, int F) { return (long long)rint(ldexp(v, F)); }

__host__ __device__ inline double fix_value(long long s, int F) { return ldexp((double)s, -F); }

__device__ inline unsigned long long lanemask_lt() {
  return (1ull << __lane_id()) - 1ull;
}

#endif  // __HIPCC__

}  // namespace kd

#define KD_HIP(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) return e_;               \
  } while (0)
