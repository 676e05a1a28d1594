// C ABI entry points (include/kd.h): argument checks, device memory, and the
// order in which the kernels of each call are enqueued.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <chrono>
#include <mutex>
#include <new>

#include "kd_internal.h"
#include "worklist.h"

using namespace kd;

// ------------------------------------------------------------------ pool

namespace kd {

static size_t size_class(size_t b) {
  if (b < 256) b = 256;
  if (b <= (1u << 20)) {
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
  }
  const size_t m = 2u << 20;
  return (b + m - 1) / m * m;
}

// A cached block of the smallest class that holds the request, up to twice
// its class (calls whose sizes vary from one to the next, as a server's
// batches do, then reuse blocks instead of allocating new ones).
void *Pool::alloc(size_t bytes) {
  const size_t c = size_class(bytes);
  {
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = free_.lower_bound(c); it != free_.end() && it->first <= 2 * c; ++it) {
      if (it->second.empty()) continue;
      void *p = it->second.back();
      it->second.pop_back();
      live_ += it->first;
      return p;
    }
  }
  void *p = nullptr;
  if (hipMalloc(&p, c) != hipSuccess) {
    (void)hipGetLastError();
    // release cached blocks and retry once
    std::lock_guard<std::mutex> g(mu_);
    for (auto &kv : free_)
      for (void *q : kv.second) {
        (void)hipFree(q);
        size_.erase(q);
      }
    free_.clear();
    if (hipMalloc(&p, c) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> g(mu_);
  size_[p] = c;
  live_ += c;
  return p;
}

void Pool::free(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu_);
  auto it = size_.find(p);
  if (it == size_.end()) return;
  free_[it->second].push_back(p);
  live_ -= it->second;
}

Pool::~Pool() {
  for (auto &kv : size_) (void)hipFree(kv.first);
}

}  // namespace kd

// --------------------------------------------------------------- helpers

namespace {

struct Scope {  // pool blocks released at scope exit (stream order makes reuse safe)
  kd_ctx *ctx;
  std::vector<void *> blocks;
  explicit Scope(kd_ctx *c) : ctx(c) {}
  template <typename T>
  T *get(size_t count) {
    void *p = ctx->pool->alloc(sizeof(T) * (count ? count : 1));
    if (p) blocks.push_back(p);
    return static_cast<T *>(p);
  }
  ~Scope() {
    for (void *p : blocks) {
      if (ctx->rec_keep) ctx->rec_keep->push_back(p);  // a batch plan keeps its temporaries
      else ctx->pool->free(p);
    }
  }
};

// Enqueues one launch on the context's stream; while a batch plan is made
// the launch is also recorded for replay (its arguments captured by value).
template <class F>
hipError_t issue(kd_ctx *ctx, F f) {
  const hipError_t e = f(ctx->stream);
  if (e == hipSuccess && ctx->rec) ctx->rec->emplace_back(f);
  return e;
}

kd_status from_hip(hipError_t e) { return e == hipSuccess ? KD_OK : KD_EDEVICE; }

constexpr double kTuneSlack = 0.01;  // kd_autotune: shapes within 1% of the fastest time alike

// Waits for the work enqueued so far on `st` by polling an event: the
// sizing read-back of a count is short, and a blocking wait wakes the host
// tens of microseconds after the device is done.  After kSpinMs of polling
// it blocks like hipStreamSynchronize.
constexpr double kSpinMs = 2.0;
hipError_t wait_stream(kd_ctx *ctx, hipStream_t st) {
  hipError_t e = hipEventRecord(ctx->wait_ev, st);
  if (e != hipSuccess) return e;
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    e = hipEventQuery(ctx->wait_ev);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() > kSpinMs)
      return hipEventSynchronize(ctx->wait_ev);
  }
}

#define KD_TRY(x)                             \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return KD_EDEVICE;  \
  } while (0)

template <typename T>
T *set_alloc(kd_set *s, size_t count) {
  void *p = s->ctx->pool->alloc(sizeof(T) * (count ? count : 1));
  if (p) s->blocks.push_back(p);
  return static_cast<T *>(p);
}

void set_free(kd_set *s) {
  if (!s) return;
  for (void *p : s->blocks) s->ctx->pool->free(p);
  delete s;
}

kd_status map_err(uint32_t code) {
  switch (code) {
    case kErrBadResidue: return KD_EBADRESIDUE;
    case kErrShort: return KD_ESHORTSEQ;
    case kErrLong: return KD_ETOOLONG;
    default: return KD_EINVAL;
  }
}

// Records the start/end events of one stage when timing is enabled.
struct StageTimer {
  kd_ctx *ctx;
  int stage;
  hipEvent_t a = nullptr, b = nullptr;
  static hipEvent_t take(kd_ctx *c) {
    if (!c->ev_free.empty()) {
      hipEvent_t e = c->ev_free.back();
      c->ev_free.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  StageTimer(kd_ctx *c, int s) : ctx(c), stage(s) {
    if (!((ctx->timing >> s) & 1u)) return;
    a = take(ctx);
    b = take(ctx);
    if (!a || !b || hipEventRecord(a, ctx->stream) != hipSuccess) {
      (void)hipGetLastError();
      if (a) ctx->ev_free.push_back(a);
      if (b) ctx->ev_free.push_back(b);
      a = b = nullptr;
    }
  }
  void done() {
    if (!a) return;
    if (hipEventRecord(b, ctx->stream) == hipSuccess) {
      ctx->pending.push_back({stage, a, b});
    } else {
      (void)hipGetLastError();
      ctx->ev_free.push_back(a);
      ctx->ev_free.push_back(b);
    }
    a = b = nullptr;
  }
  ~StageTimer() {
    if (a) ctx->ev_free.push_back(a);
    if (b) ctx->ev_free.push_back(b);
  }
};

// Copies host data to device memory on the context's stream through a
// pinned staging buffer, so the caller's host memory may change as soon as
// this returns.
hipError_t upload(kd_ctx *ctx, void *dst, const void *src, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  kd_ctx::Staged *slot = nullptr;
  for (auto &b : ctx->staging) {
    if (b.cap < bytes) continue;
    if (b.used) {
      const hipError_t q = hipEventQuery(b.ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return q;
    }
    slot = &b;
    break;
  }
  if (!slot) {
    kd_ctx::Staged b{nullptr, std::max<size_t>(bytes, 64u << 10), nullptr, false};
    KD_HIP(hipHostMalloc(&b.p, b.cap, hipHostMallocDefault));
    if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipHostFree(b.p);
      return hipErrorOutOfMemory;
    }
    ctx->staging.push_back(b);
    slot = &ctx->staging.back();
  }
  std::memcpy(slot->p, src, bytes);
  KD_HIP(hipMemcpyAsync(dst, slot->p, bytes, hipMemcpyHostToDevice, ctx->stream));
  KD_HIP(hipEventRecord(slot->ev, ctx->stream));
  slot->used = true;
  return hipSuccess;
}

void drain_timing(kd_ctx *ctx) {
  for (auto &p : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->stage_ms[p.stage] += ms;
      ctx->stage_n[p.stage] += 1;
    }
    ctx->ev_free.push_back(p.a);
    ctx->ev_free.push_back(p.b);
  }
  ctx->pending.clear();
}

}  // namespace

// --------------------------------------------------------------- context

extern "C" kd_status kd_ctx_enable_timing(kd_ctx *ctx, int enable) {
  if (!ctx) return KD_EINVAL;
  if (enable == 0) ctx->timing = 0;
  else if (enable & KD_TIME_MASK) ctx->timing = (uint32_t)enable & ((1u << KD_NSTAGES) - 1u);
  else ctx->timing = (1u << KD_NSTAGES) - 1u;
  return KD_OK;
}

extern "C" kd_status kd_ctx_stage_time(kd_ctx *ctx, int stage, double *ms, uint64_t *launches) {
  if (!ctx || stage < 0 || stage >= KD_NSTAGES) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  drain_timing(ctx);
  if (ms) *ms = ctx->stage_ms[stage];
  if (launches) *launches = ctx->stage_n[stage];
  return KD_OK;
}

extern "C" kd_status kd_ctx_reset_timing(kd_ctx *ctx) {
  if (!ctx) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  drain_timing(ctx);
  for (int i = 0; i < KD_NSTAGES; i++) {
    ctx->stage_ms[i] = 0;
    ctx->stage_n[i] = 0;
  }
  return KD_OK;
}

// Working memory of sample_partition_noalloc: one fixed array per GPU in
// the code object.  In host code `noalloc::scratch` only names the symbol;
// its device address on each GPU comes from hipGetSymbolAddress, taken once
// per device (with that device current) when the first context is created
// there, and every use goes through that address.
namespace kd {
namespace noalloc {
static_assert(KD_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) char scratch[KD_NOALLOC_SCRATCH_BYTES];
static std::mutex mu;
static std::map<int, void *> addr;  // device -> device address of its copy
}  // namespace noalloc
}  // namespace kd

namespace {

// Device address of `device`'s copy of the array; resolved on first use,
// with `device` current (the caller has set it).  nullptr on a HIP error.
void *noalloc_scratch_resolve(int device) {
  std::lock_guard<std::mutex> lk(noalloc::mu);
  auto it = noalloc::addr.find(device);
  if (it != noalloc::addr.end()) return it->second;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc::scratch)) != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return nullptr;
  }
  noalloc::addr[device] = ptr;
  return ptr;
}

}  // namespace

extern "C" kd_status kd_ctx_create(int device, void *hip_stream, kd_ctx **out) {
  if (!out) return KD_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return KD_EINVAL;
  KD_TRY(hipSetDevice(device));
  kd_ctx *c = new (std::nothrow) kd_ctx;
  if (!c) return KD_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;  // NULL: the null stream
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->cus = cus;
  if (noalloc_scratch_resolve(device) == nullptr) {
    delete c;
    return KD_EDEVICE;
  }
  c->pool = new kd::Pool();
  if (hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    delete c->pool;
    delete c;
    return KD_EDEVICE;
  }
  if (hipEventCreateWithFlags(&c->wait_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(c->pinned);
    delete c->pool;
    delete c;
    return KD_EDEVICE;
  }
  *out = c;
  return KD_OK;
}

extern "C" void kd_ctx_destroy(kd_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  drain_timing(ctx);
  for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
  for (auto &b : ctx->staging) {
    (void)hipEventDestroy(b.ev);
    (void)hipHostFree(b.p);
  }
  delete ctx->pool;  // frees task lists and anything still live
  if (ctx->wait_ev) (void)hipEventDestroy(ctx->wait_ev);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->readback) (void)hipHostFree(ctx->readback);
  delete ctx;
}

extern "C" const char *kd_strerror(kd_status s) {
  switch (s) {
    case KD_OK: return "ok";
    case KD_EINVAL: return "invalid argument";
    case KD_EBADRESIDUE: return "residue outside the 20 standard amino acids";
    case KD_ESHORTSEQ: return "sequence shorter than k = 6";
    case KD_ETOOLONG: return "sequence with more than 65535 k-mers";
    case KD_ENOMEM: return "out of device memory";
    case KD_EBUSY: return "HBM budget exhausted";
    case KD_EDEVICE: return "HIP runtime error";
    case KD_ECANCELLED: return "cancelled";
    case KD_ETOOLARGE: return "input larger than the call's fixed maximum";
    default: return "unknown status";
  }
}

extern "C" kd_status kd_last_error_info(const kd_ctx *ctx, uint64_t *seq, uint64_t *pos) {
  if (!ctx) return KD_EINVAL;
  if (seq) *seq = ctx->err_seq;
  if (pos) *pos = ctx->err_pos;
  return KD_OK;
}

extern "C" kd_status kd_ctx_synchronize(kd_ctx *ctx) {
  if (!ctx) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  return from_hip(hipStreamSynchronize(ctx->stream));
}

extern "C" void *kd_ctx_stream(kd_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

// ------------------------------------------------------------ kmer_count

namespace {

// size class of a counted object for the tuned work-list shape
uint32_t shape_class(uint32_t nsets, uint32_t N) {
  uint32_t c = 0;
  while ((2u << c) <= N) c++;
  return (nsets > 1 ? 32u : 0u) + c;
}

uint32_t tasks_per_cu(const kd_ctx *ctx, uint32_t nsets, uint32_t N) {
  auto it = ctx->tpc_pref.find(shape_class(nsets, N));
  return it != ctx->tpc_pref.end() ? it->second : kTasksPerCu;
}

void *readback_area(kd_ctx *ctx, size_t bytes);

// Counts every set of a batch (set s = sequences first[s] .. first[s+1]-1
// of the input) and lays all of them out in one pass of each kernel.  With
// a parent, the single set is made of the parent's sequences picks[0..N)
// (device input indices, all distinct) instead: their lists are taken from
// the parent, which must outlive the set, and no rank work list is built.
kd_status build_sets(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                     uint32_t nsets, const uint32_t *first, uint64_t n_residues, kd_set **out,
                     const kd_set *parent = nullptr, const uint32_t *picks = nullptr) {
  *out = nullptr;
  const uint32_t N = first[nsets];
  if (parent && (nsets != 1 || !picks)) return KD_EINVAL;
  if (!parent && N > 0 && (!offsets || (!residues && n_residues > 0))) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  kd_set *s = new (std::nothrow) kd_set;
  if (!s) return KD_ENOMEM;
  s->ctx = ctx;
  s->nsets = nsets;
  s->seq_first.assign(first, first + nsets + 1);
  s->grp_first.assign(nsets + 1, 0);
  s->rb_first.assign(nsets + 1, 0);
  for (uint32_t q = 0; q < nsets; q++) {
    const uint32_t n = first[q + 1] - first[q];
    s->grp_first[q + 1] = s->grp_first[q] + (n + 63) / 64;
    s->rb_first[q + 1] = s->rb_first[q] + (n + 15) / 16;
  }
  s->v.N = N;
  s->v.G = s->grp_first[nsets];
  s->v.RB = s->rb_first[nsets];
  s->v.base = 0;
  s->views.assign(nsets, SetView{});
  for (uint32_t q = 0; q < nsets; q++) {
    const uint32_t n = first[q + 1] - first[q];
    s->views[q].N = n;
    s->views[q].G = (n + 63) / 64;
    s->views[q].RB = (n + 15) / 16;
    s->views[q].base = first[q];
  }
  if (N == 0) {
    *out = s;
    return KD_OK;
  }
  const hipStream_t st = ctx->stream;
  const uint32_t G = s->v.G, RB = s->v.RB;
  const uint64_t cap = parent ? parent->cap : n_residues >= 5ull * N ? n_residues - 5ull * N : 0;
  Scope tmp(ctx);
  // set-owned arrays
  uint64_t *in_off = set_alloc<uint64_t>(s, N + 1);
  uint16_t *cap_ids = parent ? parent->cap_ids : set_alloc<uint16_t>(s, cap);
  uint16_t *cap_cnt = parent ? parent->cap_cnt : set_alloc<uint16_t>(s, cap);
  uint32_t *hi_cap = tmp.get<uint32_t>(cap);
  uint32_t *Dorig = set_alloc<uint32_t>(s, N);
  uint32_t *perm = set_alloc<uint32_t>(s, N);
  uint32_t *inv = set_alloc<uint32_t>(s, N);
  uint32_t *K = set_alloc<uint32_t>(s, N);
  uint32_t *D = set_alloc<uint32_t>(s, N);
  double *invK = set_alloc<double>(s, N);
  uint32_t *hi_off = set_alloc<uint32_t>(s, N + 1);
  uint64_t *grp_off = set_alloc<uint64_t>(s, G + 1);
  uint32_t *grp_len = set_alloc<uint32_t>(s, G);
  uint64_t *ghi_off = set_alloc<uint64_t>(s, G + 1);
  uint32_t *ghi_len = set_alloc<uint32_t>(s, G);
  uint32_t *exc_off = set_alloc<uint32_t>(s, RB + 1);
  uint32_t *exc_n = set_alloc<uint32_t>(s, RB);
  long long *acc = set_alloc<long long>(s, N);
  uint32_t *qhead = set_alloc<uint32_t>(s, kXcdQueues);
  uint32_t *segb = set_alloc<uint32_t>(s, 3ull * (nsets + 1));
  uint32_t *segid = nsets > 1 ? set_alloc<uint32_t>(s, (uint64_t)N + G + RB) : nullptr;

  // temporaries
  uint32_t *Korig = tmp.get<uint32_t>(N);
  uint32_t *hcount = tmp.get<uint32_t>(N);
  uint32_t *nhi_orig = tmp.get<uint32_t>(N);
  uint32_t *long_list = tmp.get<uint32_t>(N);
  uint32_t *mid_list = tmp.get<uint32_t>(N);
  uint32_t max_n = 0;
  for (uint32_t q = 0; q < nsets; q++) max_n = std::max(max_n, first[q + 1] - first[q]);
  void *sort_tmp = tmp.get<char>(sort_scratch_bytes(max_n));
  // [0] err, [1] nlong | nmid, [2] the bitmap pass's chunk counter, [8 ..]
  // LayoutMeta: cleared by one launch
  unsigned long long *small = tmp.get<unsigned long long>(8 + (sizeof(LayoutMeta) + 7) / 8);
  LayoutMeta *meta = reinterpret_cast<LayoutMeta *>(small + 8);
  void *meta_tmp = tmp.get<char>(layout_meta_scratch_bytes(N, G, RB));
  if (!in_off || !cap_ids || !cap_cnt || !hi_cap || !Dorig || !perm || !inv || !K || !D || !invK || !hi_off || !hcount ||
      !grp_off || !grp_len || !ghi_off || !ghi_len || !exc_off || !exc_n || !acc || !qhead || !segb || (nsets > 1 && !segid) ||
      !Korig || !nhi_orig || !long_list || !mid_list || !sort_tmp || !small || !meta || !meta_tmp) {
    set_free(s);
    return KD_ENOMEM;
  }
  std::vector<uint32_t> hb;
  hb.insert(hb.end(), s->seq_first.begin(), s->seq_first.end());
  hb.insert(hb.end(), s->grp_first.begin(), s->grp_first.end());
  hb.insert(hb.end(), s->rb_first.begin(), s->rb_first.end());
  Segs &sg = s->segs;
  sg.nsets = nsets;
  sg.seq = segb;
  sg.grp = segb + (nsets + 1);
  sg.rb = segb + 2 * (nsets + 1);
  sg.pos_set = segid;
  sg.grp_set = segid ? segid + N : nullptr;
  sg.rb_set = segid ? segid + N + G : nullptr;
  unsigned long long *err = small;
  uint32_t *nlong = reinterpret_cast<uint32_t *>(small + 1);  // [0] long, [1] mid
  uint32_t *nmid = nlong + 1;
  uint32_t *next_chunk = reinterpret_cast<uint32_t *>(small + 2);
  hipError_t e = upload(ctx, segb, hb.data(), sizeof(uint32_t) * hb.size());
  if (e == hipSuccess && nsets > 1)
    e = issue(ctx, [=](hipStream_t q) { return launch_seg_ids(q, sg, segid, segid + N, segid + N + G); });
  if (e == hipSuccess) {
    FillJobs f{};
    f.j[0] = {small, 1, ~0ull};
    f.j[1] = {small + 1, 7 + (sizeof(LayoutMeta) + 7) / 8, 0ull};
    f.j[2] = {reinterpret_cast<unsigned long long *>(acc), (uint64_t)N, 0ull};  // rank accumulators
    f.j[3] = {reinterpret_cast<unsigned long long *>(qhead), kXcdQueues / 2, 0ull};  // rank queues
    f.n = 4;
    e = issue(ctx, [=](hipStream_t q) { return launch_fills(q, f); });
  }
  StageTimer t_count(ctx, KD_STAGE_COUNT);
  if (e == hipSuccess && parent)
    e = launch_gather_samples(st, parent->segs, parent->in_off, parent->Dorig, picks, N, in_off, Dorig,
                              Korig, nhi_orig, hi_cap);  // (sample sets are not made under a plan)
  else if (e == hipSuccess)
    e = issue(ctx, [=](hipStream_t q) {
      return launch_count(q, residues, offsets, in_off, N, n_residues, cap, cap_ids, cap_cnt, hi_cap, Dorig,
                          Korig, nhi_orig, mid_list, nmid, long_list, nlong, next_chunk, err, ctx->cus);
    });
  t_count.done();
  StageTimer t_layout(ctx, KD_STAGE_LAYOUT);
  const std::vector<uint32_t> first_h(first, first + nsets + 1);
  if (e == hipSuccess)
    e = issue(ctx, [=](hipStream_t q) { return launch_sort_u32_index(q, Dorig, sg, first_h.data(), perm, sort_tmp); });
  if (e == hipSuccess)
    e = issue(ctx, [=](hipStream_t q) {
      return launch_layout_meta(q, sg, N, G, RB, perm, Dorig, Korig, nhi_orig, inv, K, D, invK, hcount, hi_off,
                                grp_off, grp_len, ghi_off, ghi_len, exc_off, err, meta, meta_tmp);
    });
  t_layout.done();
  // the padded list lengths come back with the totals: the rank work list
  // is cut by their estimated cost
  LayoutMeta *hm = static_cast<LayoutMeta *>(ctx->pinned);
  uint32_t *h_len = nullptr;
  if (!parent && G > 0) {
    h_len = static_cast<uint32_t *>(readback_area(ctx, 4ull * G));
    if (!h_len) {
      (void)hipStreamSynchronize(st);
      set_free(s);
      return KD_ENOMEM;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h_len, grp_len, 4ull * G, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hm, meta, sizeof(LayoutMeta), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = wait_stream(ctx, st);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    set_free(s);
    return KD_EDEVICE;
  }
  if (hm->err != ~0ull) {
    ctx->err_seq = hm->err >> 32;
    ctx->err_pos = hm->err & ((1ull << 28) - 1);
    const uint32_t code = (uint32_t)((hm->err >> 28) & 0xF);
    set_free(s);
    return map_err(code);
  }
  // the rank work list is cut on the host while the device lays the lists
  // out (below); its size is bounded by max_pair_tasks
  uint64_t task_cap = 0;
  if (!parent) {
    s->h_grp_len.assign(h_len, h_len + G);
    task_cap = max_pair_tasks(s->views, tasks_per_cu(ctx, nsets, N), ctx->cus);
  }
  s->entries = hm->entries;
  s->cap = cap;
  s->n_hi = hm->n_hi;
  s->n_gids = hm->n_gids;
  s->n_exc = hm->n_exc;
  uint16_t *gids = set_alloc<uint16_t>(s, s->n_gids + kGidsSlack);
  uint16_t *hi_ids = set_alloc<uint16_t>(s, s->n_hi);
  uint16_t *hi_cnt = set_alloc<uint16_t>(s, s->n_hi);
  uint16_t *exc_ids = set_alloc<uint16_t>(s, s->n_exc);
  uint16_t *exc_cnt = set_alloc<uint16_t>(s, 16ull * s->n_exc);
  uint32_t *ghi = set_alloc<uint32_t>(s, hm->n_ghi + 2);
  // per-set views, then (batches) the rank work list: one upload
  const size_t view_bytes = (sizeof(SetView) * nsets + 255) & ~(size_t)255;
  const size_t task_bytes = sizeof(PairTask) * (size_t)(task_cap + 1);
  char *vt = set_alloc<char>(s, view_bytes + task_bytes);
  if (!gids || !hi_ids || !hi_cnt || !exc_ids || !exc_cnt || !ghi || !vt) {
    set_free(s);
    return KD_ENOMEM;
  }
  SetView &v = s->v;
  v.perm = perm;
  v.inv = inv;
  v.K = K;
  v.D = D;
  v.invK = invK;
  v.grp_off = grp_off;
  v.grp_len = grp_len;
  v.gids = gids;
  v.hi_off = hi_off;
  v.hi_ids = hi_ids;
  v.hi_cnt = hi_cnt;
  v.ghi = ghi;
  v.ghi_off = ghi_off;
  v.ghi_len = ghi_len;
  v.exc_off = exc_off;
  v.exc_n = exc_n;
  v.exc_ids = exc_ids;
  v.exc_cnt = exc_cnt;
  v.acc = acc;
  s->queues.head = qhead;
  for (uint32_t q = 0; q < nsets; q++) {
    SetView &w = s->views[q];
    const uint32_t a = first[q], ga = s->grp_first[q], ra = s->rb_first[q];
    w.perm = perm + a;
    w.inv = inv + a;
    w.K = K + a;
    w.D = D + a;
    w.invK = invK + a;
    w.grp_off = grp_off + ga;
    w.grp_len = grp_len + ga;
    w.gids = gids;
    w.hi_off = hi_off + a;
    w.hi_ids = hi_ids;
    w.hi_cnt = hi_cnt;
    w.ghi = ghi;
    w.ghi_off = ghi_off + ga;
    w.ghi_len = ghi_len + ga;
    w.exc_off = exc_off + ra;
    w.exc_n = exc_n + ra;
    w.exc_ids = exc_ids;
    w.exc_cnt = exc_cnt;
    w.acc = acc + a;
  }
  s->cap_ids = cap_ids;
  s->cap_cnt = cap_cnt;
  s->Dorig = Dorig;
  s->in_off = in_off;
  SetView *d_view = reinterpret_cast<SetView *>(vt);
  s->d_view = d_view;
  sg.views = d_view;
  s->tasks = reinterpret_cast<PairTask *>(vt + view_bytes);
  StageTimer t_fill(ctx, KD_STAGE_LAYOUT);
  e = upload(ctx, vt, s->views.data(), sizeof(SetView) * nsets);
  if (e == hipSuccess) {
    // sentinel slack after the last group (the pair kernel reads ahead into
    // it) and the zero padding of the grouped count>=2 lists
    FillJobs f{};
    f.j[0] = {reinterpret_cast<unsigned long long *>(gids + s->n_gids), kGidsSlack / 4, 0xB640B640B640B640ull};
    f.j[1] = {reinterpret_cast<unsigned long long *>(ghi), (hm->n_ghi + 1) / 2, 0ull};
    f.n = 2;
    e = issue(ctx, [=](hipStream_t q) { return launch_fills(q, f); });
  }
  if (e == hipSuccess)
  {
    const SetView vv = v;
    const uint32_t ml = (uint32_t)hm->max_len;
    if (e == hipSuccess)
      e = issue(ctx, [=](hipStream_t q) {
        return launch_layout_fill(q, sg, vv, in_off, cap_ids, hi_cap, gids, hi_ids, hi_cnt, ghi, ml);
      });
  }
  if (e == hipSuccess)
    e = issue(ctx, [=](hipStream_t q) { return launch_exc_build(q, sg, RB, nullptr, exc_off, exc_n, exc_ids, exc_cnt); });
  t_fill.done();
  if (e == hipSuccess && !parent) {
    build_costed_tasks(s->views, s->grp_first, s->h_grp_len, tasks_per_cu(ctx, nsets, N), ctx->cus,
                       s->h_tasks, s->queues.beg);
    s->ntasks = (uint32_t)s->h_tasks.size();
    if (s->ntasks > task_cap) e = hipErrorInvalidValue;  // not expected: bounded above
    else if (s->ntasks) e = upload(ctx, s->tasks, s->h_tasks.data(), sizeof(PairTask) * s->ntasks);
  }
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    set_free(s);
    return KD_EDEVICE;
  }
  *out = s;
  return KD_OK;
}

}  // namespace

extern "C" kd_status kmer_count(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                                uint32_t n_seqs, uint64_t n_residues, kd_set **out) {
  if (!ctx || !out) return KD_EINVAL;
  *out = nullptr;
  const uint32_t first[2] = {0u, n_seqs};
  return build_sets(ctx, residues, offsets, 1, first, n_residues, out);
}

extern "C" kd_status kmer_count_batch(kd_ctx *ctx, const uint8_t *residues,
                                      const uint64_t *offsets, uint64_t n_residues,
                                      uint32_t nsets, const uint32_t *set_first, kd_set **out) {
  if (!ctx || !out) return KD_EINVAL;
  *out = nullptr;
  if (nsets == 0 || !set_first || set_first[0] != 0) return KD_EINVAL;
  for (uint32_t q = 0; q < nsets; q++)
    if (set_first[q + 1] < set_first[q]) return KD_EINVAL;
  return build_sets(ctx, residues, offsets, nsets, set_first, n_residues, out);
}

extern "C" kd_status kmer_count_blocks(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                                       uint32_t n_seqs, uint64_t n_residues, uint32_t B, kd_set **out) {
  if (!ctx || !out) return KD_EINVAL;
  *out = nullptr;
  if (B == 0 || B > n_seqs) return KD_EINVAL;
  // Algorithm 2 step 1: block b = [floor(b n / B), floor((b+1) n / B))
  std::vector<uint32_t> first(B + 1);
  for (uint32_t b = 0; b <= B; b++) first[b] = (uint32_t)((uint64_t)b * n_seqs / B);
  return build_sets(ctx, residues, offsets, B, first.data(), n_residues, out);
}

extern "C" uint32_t kd_set_count(const kd_set *s) { return s ? s->nsets : 0; }

extern "C" kd_status kd_set_first(const kd_set *s, uint32_t *first) {
  if (!s || !first) return KD_EINVAL;
  std::memcpy(first, s->seq_first.data(), sizeof(uint32_t) * s->seq_first.size());
  return KD_OK;
}

extern "C" uint32_t kd_set_size(const kd_set *s) { return s ? s->v.N : 0; }
extern "C" uint64_t kd_set_entries(const kd_set *s) { return s ? s->entries : 0; }

extern "C" void kd_set_destroy(kd_set *s) {
  if (!s) return;
  (void)hipSetDevice(s->ctx->device);
  set_free(s);
}

extern "C" kd_status kd_set_export_lists(kd_ctx *ctx, const kd_set *s, uint16_t *ids,
                                         uint16_t *counts, uint64_t *off) {
  if (!ctx || !s || s->ctx != ctx || !off || (s->entries && (!ids || !counts))) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  return from_hip(launch_export_lists(ctx->stream, s, ids, counts, off));
}

extern "C" kd_status kd_set_export_dense(kd_ctx *ctx, const kd_set *s, uint32_t first,
                                         uint32_t count, uint16_t *out) {
  if (!ctx || !s || s->ctx != ctx || (uint64_t)first + count > s->v.N || (count && !out))
    return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  return from_hip(launch_export_dense(ctx->stream, s, first, count, out));
}

// ------------------------------------------------------- kmer_similarity

extern "C" kd_status kmer_similarity(kd_ctx *ctx, const kd_set *s, uint32_t r0, uint32_t nr,
                                     uint32_t c0, uint32_t nc, uint16_t *shared, uint16_t *denom) {
  if (!ctx || !s || s->ctx != ctx || s->nsets != 1) return KD_EINVAL;
  const uint32_t N = s->v.N;
  if ((uint64_t)r0 + nr > N || (uint64_t)c0 + nc > N) return KD_EINVAL;
  if (nr == 0 || nc == 0) return KD_OK;
  if (!shared) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  Scope tmp(ctx);
  const uint32_t nb = (nr + 15) / 16;
  uint32_t *rowpos = tmp.get<uint32_t>(16ull * nb);
  uint32_t *colpos = tmp.get<uint32_t>((nc + 15) / 16 * 16ull);
  uint32_t *exc_off = tmp.get<uint32_t>(nb + 1);
  uint32_t *exc_n = tmp.get<uint32_t>(nb);
  uint16_t *exc_ids = tmp.get<uint16_t>(s->n_hi);
  uint16_t *exc_cnt = tmp.get<uint16_t>(16ull * s->n_hi);
  if (!rowpos || !colpos || !exc_off || !exc_n || !exc_ids || !exc_cnt) return KD_ENOMEM;
  KD_TRY(launch_map_positions(st, s->v.inv, r0, nr, rowpos));
  KD_TRY(launch_map_positions(st, s->v.inv, c0, nc, colpos));
  StageTimer t(ctx, KD_STAGE_SIMILARITY);
  KD_TRY(launch_exc_offsets(st, s->v, rowpos, nr, exc_off));
  KD_TRY(launch_exc_build(st, s->segs, nb, rowpos, exc_off, exc_n, exc_ids, exc_cnt));
  KD_TRY(launch_similarity(st, s->v, rowpos, nr, colpos, nc, exc_off, exc_n, exc_ids, exc_cnt,
                           shared, denom));
  t.done();
  return KD_OK;
}

// ------------------------------------------------------------- kmer_rank

extern "C" kd_status kmer_rank(kd_ctx *ctx, const kd_set *s, double delta, double *ranks) {
  if (!ctx || !s || s->ctx != ctx) return KD_EINVAL;
  if (!(delta > 0.0) || !std::isfinite(delta)) return KD_EINVAL;
  if (s->v.N == 0) return KD_OK;
  if (!ranks) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  // the accumulators are zero here: cleared when the set was counted and by
  // every finalize; a rank call that failed half-way leaves them dirty
  if (!s->acc_clean) {
    StageTimer t0(ctx, KD_STAGE_FINALIZE);
    KD_TRY(launch_fill_u64(st, s->v.acc, s->v.N, 0));
    KD_TRY(launch_fill_u64(st, s->queues.head, kXcdQueues / 2, 0));
    t0.done();
  }
  s->acc_clean = false;
  StageTimer t1(ctx, KD_STAGE_PAIRS);
  {
    const SetView *dv = s->d_view;
    const PairTask *tk = s->tasks;
    const uint32_t nt = s->ntasks, wg = (uint32_t)ctx->cus;
    const TaskQueues tq = s->queues;
    KD_TRY(issue(ctx, [=](hipStream_t q) { return launch_rank_pairs(q, dv, tk, nt, tq, wg, delta); }));
  }
  t1.done();
  StageTimer t2(ctx, KD_STAGE_FINALIZE);
  {
    const Segs sg = s->segs;
    const uint32_t N = s->v.N;
    uint32_t *qh = s->queues.head;
    KD_TRY(issue(ctx, [=](hipStream_t q) { return launch_rank_finalize(q, sg, N, delta, ranks, qh); }));
  }
  t2.done();
  s->acc_clean = true;
  return KD_OK;
}

// ------------------------------------------------------ kmer_rank_global

namespace {

kd_status plan_partition(uint32_t nsets, const uint32_t *first, const uint32_t *Bs,
                         std::vector<PartDesc> &desc, uint64_t &scratch);

// the most keys one set of a split batch sorts: its n, or its B(B-1) samples
uint32_t max_part_keys(const std::vector<PartDesc> &desc) {
  uint32_t m = 0;
  for (const PartDesc &d : desc) m = std::max(m, std::max(d.n, d.B * (d.B - 1)));
  return m;
}

// Pinned host area of at least `bytes`, valid until the next call; only
// reallocated while no copy into it is pending (callers synchronize first).
void *readback_area(kd_ctx *ctx, size_t bytes) {
  if (ctx->readback_cap < bytes) {
    if (ctx->readback) (void)hipHostFree(ctx->readback);
    ctx->readback = nullptr;
    ctx->readback_cap = 0;
    const size_t cap = std::max<size_t>(bytes, 64u << 10);
    if (hipHostMalloc(&ctx->readback, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
    ctx->readback_cap = cap;
  }
  return ctx->readback;
}

}  // namespace

extern "C" kd_status kmer_rank_global(kd_ctx *ctx, const kd_set *s, const double *local_ranks,
                                      uint32_t k, double delta, double *ranks, uint32_t *samples) {
  if (!ctx || !s || s->ctx != ctx || !local_ranks || !ranks) return KD_EINVAL;
  if (!(delta > 0.0) || !std::isfinite(delta)) return KD_EINVAL;
  const uint32_t N = s->v.N, nb = s->nsets;
  uint32_t wmin = N;
  for (uint32_t q = 0; q < nb; q++) wmin = std::min(wmin, s->seq_first[q + 1] - s->seq_first[q]);
  if (N == 0 || k == 0 || k > wmin) return KD_EINVAL;
  const uint32_t S = k * nb;  // <= N
  KD_TRY(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  Scope tmp(ctx);
  StageTimer t_pick(ctx, KD_STAGE_PARTITION);
  // steps 3-4: every block in key order (local rank, index), k samples each
  uint32_t *order = tmp.get<uint32_t>(N);
  uint32_t *bucket = tmp.get<uint32_t>(N);
  uint32_t *boff = tmp.get<uint32_t>(2ull * nb);
  uint32_t *smp = samples ? samples : tmp.get<uint32_t>(S);
  if (!order || !bucket || !boff || !smp) return KD_ENOMEM;
  if (nb == 1) {
    void *scratch = tmp.get<char>(partition_scratch_bytes(N, 1));
    if (!scratch) return KD_ENOMEM;
    KD_TRY(launch_partition(st, local_ranks, N, 1, bucket, order, boff, nullptr, nullptr, scratch));
  } else {
    std::vector<uint32_t> ones(nb, 1u);
    std::vector<PartDesc> desc;
    uint64_t scratch_bytes = 0;
    const kd_status rc = plan_partition(nb, s->seq_first.data(), ones.data(), desc, scratch_bytes);
    if (rc != KD_OK) return rc;
    void *scratch = tmp.get<char>(scratch_bytes);
    PartDesc *d_desc = tmp.get<PartDesc>(nb);
    if (!scratch || !d_desc) return KD_ENOMEM;
    KD_TRY(upload(ctx, d_desc, desc.data(), sizeof(PartDesc) * nb));
    KD_TRY(launch_partition_batch(st, d_desc, nb, max_part_keys(desc), local_ranks, bucket, order, boff,
                                  nullptr, nullptr, scratch));
  }
  KD_TRY(launch_pick_samples(st, s->segs.seq, nb, k, order, smp));
  t_pick.done();
  // column group lengths for the work list, read during the sync below
  const uint32_t G = s->v.G;
  uint32_t *h_len = static_cast<uint32_t *>(readback_area(ctx, sizeof(uint32_t) * G));
  if (!h_len) return KD_ENOMEM;
  KD_TRY(hipMemcpyAsync(h_len, s->v.grp_len, sizeof(uint32_t) * G, hipMemcpyDeviceToHost, st));
  // step 5: the samples as a set of their own (rows of the cross pass);
  // this synchronizes the stream
  const uint32_t sfirst[2] = {0, S};
  kd_set *ss = nullptr;
  kd_status rc = build_sets(ctx, nullptr, nullptr, 1, sfirst, 0, &ss, s, smp);
  if (rc != KD_OK) {
    (void)hipStreamSynchronize(st);  // the read-back copy may still be pending
    return rc;
  }
  // step 6: every sequence against the samples
  std::vector<CrossTask> tl;
  std::vector<uint32_t> gperm;
  const uint32_t gpt = make_cross_tasks(h_len, G, ss->v.RB, ctx->cus, tl, gperm);
  const size_t tbytes = (sizeof(CrossTask) * tl.size() + 255) & ~(size_t)255;
  char *d_work = tmp.get<char>(tbytes + sizeof(uint32_t) * gperm.size());
  CrossTask *d_tasks = reinterpret_cast<CrossTask *>(d_work);
  const uint32_t *d_gperm = reinterpret_cast<const uint32_t *>(d_work + tbytes);
  hipError_t e = hipErrorOutOfMemory;
  if (d_work) {
    std::vector<char> hw(tbytes + sizeof(uint32_t) * gperm.size());
    std::memcpy(hw.data(), tl.data(), sizeof(CrossTask) * tl.size());
    std::memcpy(hw.data() + tbytes, gperm.data(), sizeof(uint32_t) * gperm.size());
    e = upload(ctx, d_work, hw.data(), hw.size());
  }
  if (e == hipSuccess && !s->acc_clean) e = launch_fill_u64(st, s->v.acc, N, 0);
  s->acc_clean = false;
  StageTimer t_cross(ctx, KD_STAGE_GLOBAL);
  if (e == hipSuccess)
    e = launch_rank_cross(st, s->segs, ss->d_view, d_tasks, (uint32_t)tl.size(), d_gperm, gpt,
                          delta);
  t_cross.done();
  StageTimer t_fin(ctx, KD_STAGE_FINALIZE);
  if (e == hipSuccess) e = launch_cross_finalize(st, s->segs, N, S, delta, ranks);
  t_fin.done();
  if (e == hipSuccess) s->acc_clean = true;
  kd_set_destroy(ss);  // its blocks return to the pool; stream order keeps them valid
  if (!d_work) return KD_ENOMEM;
  return from_hip(e);
}

// ------------------------------------------------------------ decompose

extern "C" kd_status kd_decompose(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                                  uint32_t n_seqs, uint64_t n_residues, uint32_t B, int mode,
                                  double delta, double *ranks, uint32_t *bucket, uint32_t *order,
                                  uint32_t *bucket_offsets) {
  if (!ctx || !ranks || !bucket || !order || !bucket_offsets) return KD_EINVAL;
  if (mode != KD_RANK_CENTRALIZED && mode != KD_RANK_GLOBALIZED) return KD_EINVAL;
  if (n_seqs == 0 || B == 0 || B > n_seqs || B > kMaxBuckets) return KD_EINVAL;
  kd_set *s = nullptr;
  kd_status rc;
  if (mode == KD_RANK_CENTRALIZED) {
    rc = kmer_count(ctx, residues, offsets, n_seqs, n_residues, &s);
    if (rc == KD_OK) rc = kmer_rank(ctx, s, delta, ranks);
  } else {
    rc = kmer_count_blocks(ctx, residues, offsets, n_seqs, n_residues, B, &s);
    Scope tmp(ctx);
    double *local = rc == KD_OK ? tmp.get<double>(n_seqs) : nullptr;
    if (rc == KD_OK && !local) rc = KD_ENOMEM;
    if (rc == KD_OK) rc = kmer_rank(ctx, s, delta, local);
    if (rc == KD_OK) rc = kmer_rank_global(ctx, s, local, B > 1 ? B - 1 : 1, delta, ranks, nullptr);
  }
  if (s) kd_set_destroy(s);  // stream order keeps its blocks valid for the launches above
  if (rc != KD_OK) return rc;
  return sample_partition(ctx, ranks, n_seqs, B, bucket, order, bucket_offsets, nullptr, nullptr);
}

// ------------------------------------------------ buckets and guide trees

extern "C" kd_status kd_gather_sequences(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                                         uint32_t n_seqs, uint64_t n_residues, const uint32_t *order,
                                         uint32_t n, uint8_t *out_residues, uint64_t out_capacity,
                                         uint64_t *out_offsets) {
  if (!ctx || !offsets || !out_offsets || (n > 0 && !order)) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  Scope tmp(ctx);
  unsigned long long *err = tmp.get<unsigned long long>(1);
  if (!err) return KD_ENOMEM;
  StageTimer t(ctx, KD_STAGE_GATHER);
  KD_TRY(launch_fill_u64(st, err, 1, ~0ull));
  // sizes first (no bytes move while the capacity is unchecked)
  KD_TRY(launch_gather(st, residues, offsets, n_seqs, n_residues, order, n, nullptr, 0, out_offsets,
                       err));
  unsigned long long *hm = static_cast<unsigned long long *>(ctx->pinned);
  KD_TRY(hipMemcpyAsync(hm, err, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  KD_TRY(hipMemcpyAsync(hm + 1, out_offsets + n, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  KD_TRY(hipStreamSynchronize(st));
  if (hm[0] != ~0ull || hm[1] > out_capacity) return KD_EINVAL;
  if (hm[1] > 0 && (!residues || !out_residues)) return KD_EINVAL;
  KD_TRY(launch_gather(st, residues, offsets, n_seqs, n_residues, order, n, out_residues, out_capacity,
                       out_offsets, err));
  t.done();
  return KD_OK;
}

namespace {

// first element of each set's n x n matrix; false if a count overflows
bool matrix_offsets(uint32_t nsets, const uint32_t *first, std::vector<uint64_t> &doff) {
  doff.resize(nsets + 1);
  doff[0] = 0;
  for (uint32_t q = 0; q < nsets; q++) {
    const uint64_t n = first[q + 1] - first[q];
    doff[q + 1] = doff[q] + n * n;
  }
  return true;
}

}  // namespace

extern "C" kd_status kmer_distance_matrices(kd_ctx *ctx, const kd_set *s, double delta, double *dist) {
  if (!ctx || !s || s->ctx != ctx) return KD_EINVAL;
  if (!(delta > 0.0) || !std::isfinite(delta)) return KD_EINVAL;
  if (s->v.N == 0) return KD_OK;
  if (!dist) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  std::vector<uint64_t> doff;
  matrix_offsets(s->nsets, s->seq_first.data(), doff);
  // the sorted-order scratch matrices: rows rounded up to whole lines
  std::vector<uint64_t> offs(2 * s->nsets);
  uint64_t stot = 0;
  uint32_t max_n = 0;
  for (uint32_t q = 0; q < s->nsets; q++) {
    const uint64_t n = s->seq_first[q + 1] - s->seq_first[q];
    offs[q] = stot;
    offs[s->nsets + q] = doff[q];
    stot += n * ((n + 15) & ~(uint64_t)15);
    max_n = std::max(max_n, (uint32_t)n);
  }
  // its own work list: one row block per workgroup (the pair terms are
  // stored, so there are no accumulators whose flush a longer run would
  // share), the largest first
  std::vector<PairTask> tl;
  build_task_list(s->views, 1, tl);
  Scope tmp(ctx);
  uint64_t *d_off = tmp.get<uint64_t>(2 * s->nsets);
  PairTask *d_tasks = tmp.get<PairTask>(tl.size() + 1);
  double *scratch = tmp.get<double>(std::max<uint64_t>(stot, 1));
  if (!d_off || !d_tasks || !scratch) return KD_ENOMEM;
  KD_TRY(upload(ctx, d_off, offs.data(), sizeof(uint64_t) * 2 * s->nsets));
  if (!tl.empty()) KD_TRY(upload(ctx, d_tasks, tl.data(), sizeof(PairTask) * tl.size()));
  StageTimer t(ctx, KD_STAGE_DIST);
  KD_TRY(launch_distances(ctx->stream, s->segs, s->v.N, max_n, s->d_view, d_tasks, (uint32_t)tl.size(), d_off,
                          d_off + s->nsets, delta, scratch, dist));
  t.done();
  return KD_OK;
}

extern "C" kd_status upgma_trees(kd_ctx *ctx, uint32_t nsets, const uint32_t *set_first,
                                 const double *dist, int32_t *merges, double *heights) {
  if (!ctx || !set_first || nsets == 0 || !dist) return KD_EINVAL;
  if (set_first[0] != 0) return KD_EINVAL;
  uint32_t max_n = 0;
  for (uint32_t q = 0; q < nsets; q++) {
    const uint32_t n = set_first[q + 1] - set_first[q];
    if (set_first[q + 1] <= set_first[q] || n > kTreeMaxSeqs) return KD_EINVAL;
    max_n = std::max(max_n, n);
  }
  const uint32_t N = set_first[nsets];
  if (N > nsets && (!merges || !heights)) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  std::vector<uint64_t> doff;
  matrix_offsets(nsets, set_first, doff);
  Scope tmp(ctx);
  const size_t hb = sizeof(uint64_t) * nsets + sizeof(uint32_t) * (nsets + 1);
  char *d_meta = tmp.get<char>(hb);
  double *work = tmp.get<double>(doff[nsets]);
  double *rmin = tmp.get<double>(N);
  uint32_t *rarg = tmp.get<uint32_t>(N);
  unsigned long long *err = tmp.get<unsigned long long>(1);
  if (!d_meta || !work || !rmin || !rarg || !err) return KD_ENOMEM;
  std::vector<char> h(hb);
  std::memcpy(h.data(), doff.data(), sizeof(uint64_t) * nsets);
  std::memcpy(h.data() + sizeof(uint64_t) * nsets, set_first, sizeof(uint32_t) * (nsets + 1));
  KD_TRY(upload(ctx, d_meta, h.data(), hb));
  const uint64_t *d_off = reinterpret_cast<const uint64_t *>(d_meta);
  const uint32_t *d_first = reinterpret_cast<const uint32_t *>(d_meta + sizeof(uint64_t) * nsets);
  StageTimer t(ctx, KD_STAGE_TREE);
  KD_TRY(launch_fill_u64(st, err, 1, ~0ull));
  KD_TRY(hipMemcpyAsync(work, dist, sizeof(double) * doff[nsets], hipMemcpyDeviceToDevice, st));
  KD_TRY(launch_upgma(st, nsets, N, max_n, d_first, d_off, work, rmin, rarg, merges, heights, err));
  t.done();
  unsigned long long *hm = static_cast<unsigned long long *>(ctx->pinned);
  KD_TRY(hipMemcpyAsync(hm, err, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  KD_TRY(hipStreamSynchronize(st));
  return hm[0] == ~0ull ? KD_OK : KD_EINVAL;
}

// ------------------------------------------------- profiles and PSP scores

extern "C" kd_status psp_profile(kd_ctx *ctx, const uint8_t *aln, uint32_t m, uint32_t L, double *f) {
  if (!ctx || m == 0) return KD_EINVAL;
  if (L == 0) return KD_OK;
  if (!aln || !f) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  Scope tmp(ctx);
  unsigned long long *bad = tmp.get<unsigned long long>(1);
  if (!bad) return KD_ENOMEM;
  StageTimer t(ctx, KD_STAGE_PSP);
  KD_TRY(launch_fill_u64(st, bad, 1, ~0ull));
  KD_TRY(launch_psp_profile(st, aln, m, L, f, bad));
  t.done();
  unsigned long long *hm = static_cast<unsigned long long *>(ctx->pinned);
  KD_TRY(hipMemcpyAsync(hm, bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  KD_TRY(hipStreamSynchronize(st));
  if (hm[0] != ~0ull) {
    ctx->err_seq = hm[0] / L;
    ctx->err_pos = hm[0] % L;
    return KD_EBADRESIDUE;
  }
  return KD_OK;
}

extern "C" kd_status psp_scores(kd_ctx *ctx, const double *M, uint32_t npairs, const kd_psp_pair *pairs) {
  if (!ctx || !M || (npairs > 0 && !pairs)) return KD_EINVAL;
  // descriptors of the pairs that have scores, with their grid offsets
  std::vector<PspWork> h;
  uint64_t gsz = 0, gblks = 0, tiles = 0;
  for (uint32_t q = 0; q < npairs; q++) {
    const kd_psp_pair &p = pairs[q];
    if (p.lx == 0 || p.ly == 0) continue;  // empty pairs write nothing
    if (!p.fx || !p.fy || !p.scores) return KD_EINVAL;
    h.push_back(PspWork{p.fx, p.fy, p.scores, nullptr, p.lx, p.ly, 0, 0});
    gsz += 20ull * p.lx;
  }
  if (h.empty()) return KD_OK;
  if (!psp_plan(h, gblks, tiles)) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  Scope tmp(ctx);
  PspWork *d_w = tmp.get<PspWork>(h.size());
  double *g = tmp.get<double>(gsz);
  if (!d_w || !g) return KD_ENOMEM;
  uint64_t go = 0;
  for (auto &p : h) {
    p.g = g + go;
    go += 20ull * p.lx;
  }
  KD_TRY(upload(ctx, d_w, h.data(), sizeof(PspWork) * h.size()));
  StageTimer t(ctx, KD_STAGE_PSP);
  KD_TRY(launch_psp_scores(ctx->stream, d_w, (uint32_t)h.size(), (uint32_t)gblks, (uint32_t)tiles, M));
  t.done();
  return KD_OK;
}

// ------------------------------------------------------------ autotune

extern "C" kd_status kd_autotune(kd_ctx *ctx, kd_set *s, double delta, uint32_t *best,
                                 double *ms_out) {
  if (!ctx || !s || s->ctx != ctx) return KD_EINVAL;
  if (!(delta > 0.0) || !std::isfinite(delta)) return KD_EINVAL;
  static const uint32_t cand[KD_TUNE_CANDIDATES] = {8, 16, 32, 64, 128};
  const uint32_t N = s->v.N;
  if (N == 0 || s->h_grp_len.size() != s->v.G) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  const hipStream_t st = ctx->stream;
  Scope tmp(ctx);
  double *R = tmp.get<double>(N);
  if (!R) return KD_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KD_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return KD_EDEVICE;
  }
  std::vector<double> ref(N), got(N);
  kd_status rc = KD_OK;
  double best_ms = 1e300;
  uint32_t best_tpc = kTasksPerCu;
  double avg_ms[KD_TUNE_CANDIDATES];
  for (int c = 0; c < KD_TUNE_CANDIDATES && rc == KD_OK; c++) {
    // this candidate's work list, in a block of its own
    std::vector<PairTask> tl;
    build_costed_tasks(s->views, s->grp_first, s->h_grp_len, cand[c], ctx->cus, tl, s->queues.beg);
    PairTask *d = set_alloc<PairTask>(s, tl.size() + 1);
    if (!d) {
      rc = KD_ENOMEM;
      break;
    }
    if (upload(ctx, d, tl.data(), sizeof(PairTask) * tl.size()) != hipSuccess) {
      rc = KD_EDEVICE;
      break;
    }
    s->tasks = d;
    s->ntasks = (uint32_t)tl.size();
    s->h_tasks.swap(tl);
    float ms = 0.f, tot = 0.f;
    for (int it = 0; it < 4 && rc == KD_OK; it++) {  // one warm-up, three timed
      if (hipEventRecord(e0, st) != hipSuccess) rc = KD_EDEVICE;
      if (rc == KD_OK) rc = kmer_rank(ctx, s, delta, R);
      if (rc == KD_OK && hipEventRecord(e1, st) != hipSuccess) rc = KD_EDEVICE;
      if (rc == KD_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = KD_EDEVICE;
      if (it > 0) tot += ms;
    }
    if (rc != KD_OK) break;
    const double avg = tot / 3.0;
    avg_ms[c] = avg;
    if (ms_out) ms_out[c] = avg;
    if (hipMemcpy(c == 0 ? ref.data() : got.data(), R, 8ull * N, hipMemcpyDeviceToHost) != hipSuccess) {
      rc = KD_EDEVICE;
      break;
    }
    // the accumulation is exact: every work-list shape gives the same bits
    if (c > 0 && std::memcmp(ref.data(), got.data(), 8ull * N) != 0) {
      rc = KD_EDEVICE;
      break;
    }
    best_ms = std::min(best_ms, avg);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != KD_OK) return rc;
  // the fewest tasks (fewest column flushes) within kTuneSlack of the
  // fastest: shapes that time alike would otherwise win by noise
  for (int c = KD_TUNE_CANDIDATES - 1; c >= 0; c--)
    if (avg_ms[c] <= best_ms * (1.0 + kTuneSlack)) best_tpc = cand[c];
  ctx->tpc_pref[shape_class(s->nsets, N)] = best_tpc;
  // the set keeps the winner's work list
  std::vector<PairTask> tl;
  build_costed_tasks(s->views, s->grp_first, s->h_grp_len, best_tpc, ctx->cus, tl, s->queues.beg);
  PairTask *d = set_alloc<PairTask>(s, tl.size() + 1);
  if (!d) return KD_ENOMEM;
  KD_TRY(upload(ctx, d, tl.data(), sizeof(PairTask) * tl.size()));
  s->tasks = d;
  s->ntasks = (uint32_t)tl.size();
  s->h_tasks.swap(tl);
  if (best) *best = best_tpc;
  return KD_OK;
}

extern "C" kd_status kd_ctx_set_tasks_per_cu(kd_ctx *ctx, uint32_t nsets, uint32_t n, uint32_t tasks) {
  if (!ctx || tasks == 0 || tasks > 4096) return KD_EINVAL;
  ctx->tpc_pref[shape_class(nsets, n)] = tasks;
  return KD_OK;
}

// ------------------------------------------------------ sample_partition

extern "C" kd_status sample_partition(kd_ctx *ctx, const double *ranks, uint32_t n, uint32_t B,
                                      uint32_t *bucket, uint32_t *order, uint32_t *offsets,
                                      double *pivot_rank, uint32_t *pivot_idx) {
  if (!ctx || !ranks || !bucket || !order || !offsets) return KD_EINVAL;
  if (n == 0 || B == 0 || B > n || B > kMaxBuckets) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  Scope tmp(ctx);
  void *scratch = tmp.get<char>(partition_scratch_bytes(n, B));
  if (!scratch) return KD_ENOMEM;
  StageTimer t(ctx, KD_STAGE_PARTITION);
  KD_TRY(launch_partition(ctx->stream, ranks, n, B, bucket, order, offsets, pivot_rank, pivot_idx,
                          scratch));
  t.done();
  return KD_OK;
}

extern "C" kd_status sample_partition_noalloc(kd_ctx *ctx, const double *ranks, uint32_t n,
                                              uint32_t B, uint32_t *bucket, uint32_t *order,
                                              uint32_t *offsets, double *pivot_rank,
                                              uint32_t *pivot_idx) {
  if (!ctx || !ranks || !bucket || !order || !offsets) return KD_EINVAL;
  if (n == 0 || B == 0 || B > n || B > kMaxBuckets) return KD_EINVAL;
  if (n > KD_NOALLOC_MAX_KEYS) return KD_ETOOLARGE;
  if (partition_scratch_bytes(n, B) > KD_NOALLOC_SCRATCH_BYTES) return KD_ETOOLARGE;
  KD_TRY(hipSetDevice(ctx->device));
  void *scratch_dev = nullptr;
  {
    std::lock_guard<std::mutex> lk(noalloc::mu);
    auto it = noalloc::addr.find(ctx->device);
    if (it != noalloc::addr.end()) scratch_dev = it->second;
  }
  if (!scratch_dev) return KD_EDEVICE;  // kd_ctx_create resolved it for this device
  KD_TRY(launch_partition(ctx->stream, ranks, n, B, bucket, order, offsets, pivot_rank, pivot_idx,
                          scratch_dev));
  return KD_OK;
}

namespace {

// Per-set split descriptors of a batch: where each set's keys, outputs and
// scratch start.
kd_status plan_partition(uint32_t nsets, const uint32_t *first, const uint32_t *Bs,
                         std::vector<PartDesc> &desc, uint64_t &scratch) {
  desc.resize(nsets);
  scratch = 0;
  uint64_t ob = 0, pb = 0;
  for (uint32_t q = 0; q < nsets; q++) {
    const uint32_t n = first[q + 1] - first[q], B = Bs[q];
    if (n == 0 || B == 0 || B > n || B > kMaxBuckets) return KD_EINVAL;
    desc[q].scratch_off = scratch;
    desc[q].first = first[q];
    desc[q].n = n;
    desc[q].B = B;
    desc[q].off_base = (uint32_t)ob;
    desc[q].piv_base = (uint32_t)pb;
    scratch += (partition_scratch_bytes(n, B) + 255) & ~(uint64_t)255;
    ob += B + 1;
    pb += B - 1;
  }
  return KD_OK;
}

}  // namespace

extern "C" kd_status sample_partition_batch(kd_ctx *ctx, const double *ranks, uint32_t nsets,
                                            const uint32_t *set_first, const uint32_t *set_B,
                                            uint32_t *bucket, uint32_t *order, uint32_t *offsets,
                                            double *pivot_rank, uint32_t *pivot_idx) {
  if (!ctx || !ranks || !bucket || !order || !offsets || !set_first || !set_B || nsets == 0)
    return KD_EINVAL;
  if (set_first[0] != 0) return KD_EINVAL;
  for (uint32_t q = 0; q < nsets; q++)
    if (set_first[q + 1] < set_first[q]) return KD_EINVAL;
  std::vector<PartDesc> desc;
  uint64_t scratch_bytes = 0;
  kd_status rc = plan_partition(nsets, set_first, set_B, desc, scratch_bytes);
  if (rc != KD_OK) return rc;
  KD_TRY(hipSetDevice(ctx->device));
  Scope tmp(ctx);
  void *scratch = tmp.get<char>(scratch_bytes);
  PartDesc *d_desc = tmp.get<PartDesc>(nsets);
  if (!scratch || !d_desc) return KD_ENOMEM;
  KD_TRY(upload(ctx, d_desc, desc.data(), sizeof(PartDesc) * nsets));
  StageTimer t(ctx, KD_STAGE_PARTITION);
  const uint32_t mk = max_part_keys(desc);
  KD_TRY(issue(ctx, [=](hipStream_t q) {
    return launch_partition_batch(q, d_desc, nsets, mk, ranks, bucket, order, offsets, pivot_rank, pivot_idx,
                                  scratch);
  }));
  t.done();
  return KD_OK;
}

extern "C" kd_status kd_batch_run(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                                  uint64_t n_residues, uint32_t nsets, const uint32_t *set_first,
                                  const uint32_t *set_B, double delta, double *ranks,
                                  uint32_t *bucket, uint32_t *order, uint32_t *bucket_off) {
  if (!ctx || !set_first || !set_B || nsets == 0 || !ranks || !bucket || !order || !bucket_off)
    return KD_EINVAL;
  if (!(delta > 0.0) || !std::isfinite(delta)) return KD_EINVAL;
  if (set_first[0] != 0) return KD_EINVAL;
  for (uint32_t q = 0; q < nsets; q++) {
    const uint32_t n = set_first[q + 1] - set_first[q];
    if (set_first[q + 1] < set_first[q] || set_B[q] == 0 || set_B[q] > n || set_B[q] > kMaxBuckets)
      return KD_EINVAL;
  }
  kd_set *s = nullptr;
  kd_status rc = kmer_count_batch(ctx, residues, offsets, n_residues, nsets, set_first, &s);
  if (rc != KD_OK) return rc;
  rc = kmer_rank(ctx, s, delta, ranks);
  if (rc == KD_OK)
    rc = sample_partition_batch(ctx, ranks, nsets, set_first, set_B, bucket, order, bucket_off,
                                nullptr, nullptr);
  kd_set_destroy(s);  // its blocks return to the pool; stream order keeps them valid
  return rc;
}

// ---------------------------------------------------------- batch plans

struct kd_batch_plan {
  kd_ctx *ctx = nullptr;
  kd_set *set = nullptr;
  std::vector<void *> blocks;  // input copies and the batch's temporaries (pool blocks)
  std::vector<std::function<hipError_t(hipStream_t)>> launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void plan_free(kd_batch_plan *p) {
  if (!p) return;
  kd_ctx *ctx = p->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);  // no replay may still use the blocks
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->set) kd_set_destroy(p->set);
  for (void *b : p->blocks) ctx->pool->free(b);
  delete p;
}

}  // namespace

extern "C" kd_status kd_batch_plan_create(kd_ctx *ctx, const uint8_t *residues, const uint64_t *offsets,
                                          uint64_t n_residues, uint32_t nsets, const uint32_t *set_first,
                                          const uint32_t *set_B, double delta, double *ranks,
                                          uint32_t *bucket, uint32_t *order, uint32_t *offsets_out,
                                          kd_batch_plan **out) {
  if (!out) return KD_EINVAL;
  *out = nullptr;
  if (!ctx || !set_first || !set_B || nsets == 0 || !ranks || !bucket || !order || !offsets_out)
    return KD_EINVAL;
  if (!(delta > 0.0) || !std::isfinite(delta)) return KD_EINVAL;
  if (set_first[0] != 0) return KD_EINVAL;
  for (uint32_t q = 0; q < nsets; q++) {
    const uint32_t n = set_first[q + 1] - set_first[q];
    if (set_first[q + 1] < set_first[q] || set_B[q] == 0 || set_B[q] > n || set_B[q] > kMaxBuckets)
      return KD_EINVAL;
  }
  const uint32_t N = set_first[nsets];
  if (N > 0 && (!offsets || (!residues && n_residues > 0))) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  kd_batch_plan *p = new (std::nothrow) kd_batch_plan;
  if (!p) return KD_ENOMEM;
  p->ctx = ctx;
  // the plan's own copies of the inputs: every replay reads the same batch
  uint8_t *res = static_cast<uint8_t *>(ctx->pool->alloc(std::max<uint64_t>(n_residues, 1)));
  if (res) p->blocks.push_back(res);
  uint64_t *off = static_cast<uint64_t *>(ctx->pool->alloc(8ull * (N + 1)));
  if (off) p->blocks.push_back(off);
  if (!res || !off) {
    plan_free(p);
    return KD_ENOMEM;
  }
  hipError_t e = hipMemcpyAsync(res, residues, n_residues, hipMemcpyDefault, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(off, offsets, 8ull * (N + 1), hipMemcpyDefault, ctx->stream);
  if (e != hipSuccess) {
    plan_free(p);
    return KD_EDEVICE;
  }
  // the batch once, eagerly, with every kernel launch recorded
  ctx->rec = &p->launches;
  ctx->rec_keep = &p->blocks;
  kd_status rc = kmer_count_batch(ctx, res, off, n_residues, nsets, set_first, &p->set);
  if (rc == KD_OK) rc = kmer_rank(ctx, p->set, delta, ranks);
  if (rc == KD_OK)
    rc = sample_partition_batch(ctx, ranks, nsets, set_first, set_B, bucket, order, offsets_out, nullptr,
                                nullptr);
  ctx->rec = nullptr;
  ctx->rec_keep = nullptr;
  if (rc == KD_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) rc = KD_EDEVICE;
  // the recorded launches, replayed into a graph on a capture stream of the
  // default priority
  hipStream_t cs = nullptr;
  if (rc == KD_OK && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = KD_EDEVICE;
  if (rc == KD_OK) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (size_t i = 0; e == hipSuccess && i < p->launches.size(); i++) e = p->launches[i](cs);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    p->graph = g;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      rc = KD_EDEVICE;
    }
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (rc != KD_OK) {
    plan_free(p);
    return rc;
  }
  *out = p;
  return KD_OK;
}

extern "C" kd_status kd_batch_plan_launch(kd_batch_plan *p) {
  if (!p || !p->exec) return KD_EINVAL;
  KD_TRY(hipSetDevice(p->ctx->device));
  return from_hip(hipGraphLaunch(p->exec, p->ctx->stream));
}

extern "C" uint32_t kd_batch_plan_launches(const kd_batch_plan *p) {
  if (!p || !p->graph) return 0u;
  size_t n = 0;
  if (hipGraphGetNodes(p->graph, nullptr, &n) != hipSuccess) {
    (void)hipGetLastError();
    return 0u;
  }
  return (uint32_t)n;
}

extern "C" void kd_batch_plan_destroy(kd_batch_plan *p) { plan_free(p); }

// ---------------------------------------------------------- calibration

extern "C" kd_status kd_calibrate_lds(kd_ctx *ctx, uint32_t workgroups, uint32_t steps,
                                      uint32_t batch, double *ms, uint64_t *wave_reads) {
  if (!ctx || !ms || !wave_reads || workgroups == 0 || steps == 0) return KD_EINVAL;
  if (batch != 2 && batch != 8 && batch != 32) return KD_EINVAL;
  KD_TRY(hipSetDevice(ctx->device));
  Scope tmp(ctx);
  uint32_t *sink = tmp.get<uint32_t>(1024ull * workgroups);
  if (!sink) return KD_ENOMEM;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess) return KD_EDEVICE;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return KD_EDEVICE;
  }
  kd_status rc = KD_OK;
  float t = 0.f;
  if (hipEventRecord(a, ctx->stream) != hipSuccess ||
      launch_lds_probe(ctx->stream, workgroups, steps, batch, sink) != hipSuccess ||
      hipEventRecord(b, ctx->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
      hipEventElapsedTime(&t, a, b) != hipSuccess)
    rc = KD_EDEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != KD_OK) return rc;
  *ms = t;
  *wave_reads = 16ull * workgroups * steps * 32ull;  // 16 waves per workgroup
  return KD_OK;
}
