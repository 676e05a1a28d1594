// Request server (kd_server_*): admission against a device-memory budget
// and continuous batching of independent jobs onto the batched path.
//
// One worker thread owns a context and a stream.  Jobs move
//   waiting --(fits the budget)--> admitted --(picked by a batch)--> running
//   --> done (a completion record waits for kd_server_poll).
// Whenever the worker is free it takes every admitted job with the delta
// of the oldest one (within the batch limits), concatenates them into one
// input, and runs count -> rank -> split for all of them at once; jobs
// arriving meanwhile wait for the next batch.  A job with bad input fails
// alone: the batch is re-run without it.  A job's residues go to the
// device when it is submitted (a copy stream of their own), so a batch
// finds its input there and only gathers it into one buffer.
#include <time.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <unordered_map>

#include "kd_internal.h"

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

// The server's device current for the scope, the caller's restored after.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != d) (void)hipSetDevice(d);
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

struct Job {
  uint64_t ticket = 0;
  kd_job out{};                    // caller's output pointers (inputs copied below)
  uint8_t *res = nullptr;          // the residues: in arena chunk `chunk`, or in `own`
  const uint8_t *dres = nullptr;   // their device copy (the chunk's mirror), or null
  int chunk = -1;
  std::vector<uint8_t> own;
  std::vector<uint64_t> offsets;
  uint64_t bytes = 0;              // admission charge
  uint64_t t_submit = 0, t_start = 0;
};

// Pinned host memory for the jobs' residues, so that a batch's input goes to
// the device by asynchronous DMA straight from each job's copy: chunks of
// kChunk bytes that stay with the server, bump allocation, a chunk reused
// once every job placed in it has finished.  Non-coherent pinned memory:
// the CPU writes it through its caches (the default, coherent kind was much
// slower to fill), and the device only reads it by copies issued after the
// job's data is in place.  Each chunk has a device mirror at the same
// offsets (null if device memory ran out), which the job's copy at submit
// fills.  Guarded by the server's mutex; chunks are added with the server's
// device current.
struct Arena {
  static constexpr size_t kChunk = 64ull << 20;
  struct Chunk {
    uint8_t *p = nullptr;
    uint8_t *d = nullptr;
    size_t used = 0;
    uint32_t refs = 0;
  };
  std::vector<Chunk> chunks;
  size_t cur = 0;
  bool mirrored = true;  // chunks get device mirrors
  bool add_chunk(bool touch) {
    void *v = nullptr;
    if (hipHostMalloc(&v, kChunk, hipHostMallocNonCoherent) != hipSuccess) return false;
    uint8_t *p = static_cast<uint8_t *>(v);
    if (touch) std::memset(p, 0, kChunk);
    void *d = nullptr;
    if (mirrored && hipMalloc(&d, kChunk) != hipSuccess) {
      (void)hipGetLastError();
      d = nullptr;
    }
    chunks.push_back(Chunk{p, static_cast<uint8_t *>(d), 0, 0});
    return true;
  }
  uint8_t *mirror(int k, const uint8_t *p) const {
    const Chunk &c = chunks[(size_t)k];
    return c.d ? c.d + (p - c.p) : nullptr;
  }
  // n bytes; the chunk index, or -1 when the job must hold its own copy
  int alloc(size_t n, uint8_t *&p) {
    const size_t a = (n + 255) & ~(size_t)255;
    if (n == 0 || a > kChunk) return -1;
    if (cur >= chunks.size() || chunks[cur].used + a > kChunk) {
      size_t k = 0;
      while (k < chunks.size() && chunks[k].refs) k++;  // a chunk no job uses any more
      if (k == chunks.size() && !add_chunk(false)) return -1;
      chunks[k].used = 0;
      cur = k;
    }
    Chunk &c = chunks[cur];
    p = c.p + c.used;
    c.used += a;
    c.refs++;
    return (int)cur;
  }
  void release(int k) {
    if (k >= 0 && --chunks[(size_t)k].refs == 0 && (size_t)k != cur) chunks[(size_t)k].used = 0;
  }
  ~Arena() {
    for (auto &c : chunks) {
      (void)hipHostFree(c.p);
      if (c.d) (void)hipFree(c.d);
    }
  }
};

// Pieces of the jobs' device copies to gather into a batch's input: one
// workgroup per piece of at most kPiece bytes, byte copies (the source and
// destination offsets have no common alignment), eight loads in flight per
// thread.
struct Piece {
  const uint8_t *src;
  uint64_t dst;  // byte offset in the batch's residues
  uint64_t len;  // 1 .. kPiece
};
constexpr uint64_t kPiece = 64ull << 10;

__global__ __launch_bounds__(256) void gather_pieces_kernel(const Piece *__restrict__ pieces,
                                                            uint8_t *__restrict__ out) {
  const Piece pc = pieces[blockIdx.x];
  const uint8_t *__restrict__ src = pc.src;
  uint8_t *__restrict__ dst = out + pc.dst;
  const uint32_t len = (uint32_t)pc.len;
  for (uint32_t t0 = threadIdx.x; t0 < len; t0 += 256u * 8u) {
    uint8_t v[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; u++) {
      const uint32_t t = t0 + 256u * u;
      v[u] = t < len ? src[t] : 0;
    }
#pragma unroll
    for (uint32_t u = 0; u < 8; u++) {
      const uint32_t t = t0 + 256u * u;
      if (t < len) dst[t] = v[u];
    }
  }
}

// grow-only buffers; the host ones are non-coherent pinned memory, which
// the CPU reads and writes through its caches (the batch's offsets are
// written there, its results read back from there)
struct HostBuf {
  void *p = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t n) {
    if (n <= cap) return hipSuccess;
    const size_t c = std::max(n, cap * 2);
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc(&p, c, hipHostMallocNonCoherent);
    if (e == hipSuccess) cap = c;
    return e;
  }
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
};

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t n) {
    if (n <= cap) return hipSuccess;
    const size_t c = std::max(n, cap * 2);
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(&p, c);
    if (e == hipSuccess) cap = c;
    return e;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

struct kd_server {
  int device = 0;
  kd_server_opts opts{};
  hipStream_t stream = nullptr;
  hipStream_t copy_stream = nullptr;  // the jobs' copies at submit
  hipEvent_t copy_ev = nullptr;       // recorded after each of them (under mu)
  kd_ctx *ctx = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<Job *> waiting, admitted;
  std::unordered_map<uint64_t, Job *> running;
  std::deque<kd_done> done;
  uint64_t reserved = 0;
  Arena arena;  // the jobs' residues (pinned)
  // staging, used by the worker only
  HostBuf h_in, h_out;
  DevBuf d_in, d_out;

  void admit_locked() {  // FIFO: the oldest waiting job goes first
    while (!waiting.empty() && reserved + waiting.front()->bytes <= opts.hbm_budget) {
      reserved += waiting.front()->bytes;
      admitted.push_back(waiting.front());
      waiting.pop_front();
    }
  }

  void finish_locked(Job *j, kd_status st, uint32_t batch_jobs, uint64_t t_done) {
    kd_done d{};
    d.ticket = j->ticket;
    d.status = st;
    d.batch_jobs = batch_jobs;
    d.t_submit_ns = j->t_submit;
    d.t_start_ns = j->t_start;
    d.t_done_ns = t_done;
    done.push_back(d);
    reserved -= j->bytes;
    arena.release(j->chunk);
    delete j;
  }

  kd_status run_batch(std::vector<Job *> &b, std::vector<kd_status> &st);
  void loop();
};

// Runs the jobs of b (all st[q] == KD_OK on entry) as one batch; on return
// st[q] is each job's status and its outputs are written when KD_OK.
kd_status kd_server::run_batch(std::vector<Job *> &b, std::vector<kd_status> &st) {
  for (;;) {
    std::vector<uint32_t> live;
    for (uint32_t q = 0; q < b.size(); q++)
      if (st[q] == KD_OK) live.push_back(q);
    if (live.empty()) return KD_OK;
    const uint32_t ns = (uint32_t)live.size();
    std::vector<uint32_t> first(ns + 1, 0), Bs(ns);
    uint64_t nres = 0;
    for (uint32_t k = 0; k < ns; k++) {
      const Job *j = b[live[k]];
      first[k + 1] = first[k] + j->out.n_seqs;
      Bs[k] = j->out.B;
      nres += j->out.n_residues;
    }
    const uint32_t N = first[ns];
    uint64_t nb = 0, npc = 0;
    for (uint32_t k = 0; k < ns; k++) {
      nb += Bs[k] + 1;
      const Job *j = b[live[k]];
      if (j->dres) npc += (j->out.n_residues + kPiece - 1) / kPiece;
    }
    // input: offsets (N+1 u64, rebased) and the gather pieces, staged in
    // pinned memory, then the residues (gathered from the jobs' device
    // copies; a job without one is sent from its host copy);
    // output: ranks, bucket, order, offsets
    const size_t tab_at = (8ull * (N + 1) + 15) & ~(size_t)15;
    const size_t head = tab_at + sizeof(Piece) * npc;
    const size_t in_bytes = head + nres;
    const size_t out_bytes = 8ull * N + 4ull * N + 4ull * N + 4ull * nb;
    if (h_in.reserve(head) != hipSuccess || h_out.reserve(out_bytes) != hipSuccess ||
        d_in.reserve(in_bytes) != hipSuccess || d_out.reserve(out_bytes + 256) != hipSuccess) {
      for (uint32_t q : live) st[q] = KD_ENOMEM;
      return KD_ENOMEM;
    }
    uint64_t *off = static_cast<uint64_t *>(h_in.p);
    Piece *pcs = reinterpret_cast<Piece *>(static_cast<char *>(h_in.p) + tab_at);
    uint8_t *d_resw = static_cast<uint8_t *>(d_in.p) + head;
    uint64_t r0 = 0, pq = 0;
    bool copied = true;
    for (uint32_t k = 0; k < ns; k++) {
      const Job *j = b[live[k]];
      const uint64_t n = j->out.n_residues;
      for (uint32_t i = 0; i < j->out.n_seqs; i++) off[first[k] + i] = r0 + j->offsets[i];
      if (j->dres) {
        for (uint64_t a = 0; a < n; a += kPiece) pcs[pq++] = Piece{j->dres + a, r0 + a, std::min(kPiece, n - a)};
      } else {
        copied = copied && hipMemcpyAsync(d_resw + r0, j->res, n, hipMemcpyHostToDevice, stream) == hipSuccess;
      }
      r0 += n;
    }
    off[N] = r0;
    char *dout = static_cast<char *>(d_out.p);
    double *d_ranks = reinterpret_cast<double *>(dout);
    uint32_t *d_bucket = reinterpret_cast<uint32_t *>(dout + 8ull * N);
    uint32_t *d_order = d_bucket + N;
    uint32_t *d_offs = d_order + N;
    const uint8_t *d_res = d_resw;
    const uint64_t *d_off = static_cast<const uint64_t *>(d_in.p);
    copied = copied && hipMemcpyAsync(d_in.p, h_in.p, head, hipMemcpyHostToDevice, stream) == hipSuccess;
    if (copied && npc) {
      hipLaunchKernelGGL(gather_pieces_kernel, dim3((uint32_t)npc), dim3(256), 0, stream,
                         reinterpret_cast<const Piece *>(static_cast<char *>(d_in.p) + tab_at), d_resw);
      copied = hipGetLastError() == hipSuccess;
    }
    if (!copied) {
      for (uint32_t x : live) st[x] = KD_EDEVICE;
      return KD_EDEVICE;
    }
    kd_set *set = nullptr;
    kd_status rc = kmer_count_batch(ctx, d_res, d_off, nres, ns, first.data(), &set);
    if (rc == KD_EBADRESIDUE || rc == KD_ESHORTSEQ || rc == KD_ETOOLONG) {
      // the job holding the offending sequence fails; the others run again
      uint64_t seq = 0, pos = 0;
      kd_last_error_info(ctx, &seq, &pos);
      const uint32_t k = (uint32_t)(std::upper_bound(first.begin(), first.end(), (uint32_t)seq) - first.begin()) - 1;
      st[live[std::min(k, ns - 1)]] = rc;
      continue;
    }
    if (rc == KD_OK) rc = kmer_rank(ctx, set, b[live[0]]->out.delta, d_ranks);
    if (rc == KD_OK)
      rc = sample_partition_batch(ctx, d_ranks, ns, first.data(), Bs.data(), d_bucket, d_order,
                                  d_offs, nullptr, nullptr);
    if (rc == KD_OK && hipMemcpyAsync(h_out.p, d_out.p, out_bytes, hipMemcpyDeviceToHost, stream) != hipSuccess)
      rc = KD_EDEVICE;
    if (rc == KD_OK && hipStreamSynchronize(stream) != hipSuccess) rc = KD_EDEVICE;
    if (set) kd_set_destroy(set);
    if (rc != KD_OK) {
      for (uint32_t q : live) st[q] = rc;
      return rc;
    }
    const char *hout = static_cast<const char *>(h_out.p);
    const double *h_ranks = reinterpret_cast<const double *>(hout);
    const uint32_t *h_bucket = reinterpret_cast<const uint32_t *>(hout + 8ull * N);
    const uint32_t *h_order = h_bucket + N;
    const uint32_t *h_offs = h_order + N;
    uint64_t ob = 0;
    for (uint32_t k = 0; k < ns; k++) {
      const kd_job &o = b[live[k]]->out;
      const uint32_t a = first[k], n = o.n_seqs;
      if (o.ranks) std::memcpy(o.ranks, h_ranks + a, 8ull * n);
      if (o.bucket) std::memcpy(o.bucket, h_bucket + a, 4ull * n);
      if (o.order) std::memcpy(o.order, h_order + a, 4ull * n);
      if (o.bucket_offsets) std::memcpy(o.bucket_offsets, h_offs + ob, 4ull * (o.B + 1));
      ob += o.B + 1;
    }
    return KD_OK;
  }
}

void kd_server::loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || !admitted.empty(); });
    if (stop) break;
    // the batch: admitted jobs of the oldest job's delta, in FIFO order
    const double delta = admitted.front()->out.delta;
    std::vector<Job *> b;
    uint64_t seqs = 0;
    for (auto it = admitted.begin(); it != admitted.end();) {
      Job *j = *it;
      if (opts.max_batch_jobs && b.size() >= opts.max_batch_jobs) break;
      if (j->out.delta != delta) {
        ++it;
        continue;
      }
      if (!b.empty() && opts.max_batch_seqs && seqs + j->out.n_seqs > opts.max_batch_seqs) break;
      seqs += j->out.n_seqs;
      b.push_back(j);
      it = admitted.erase(it);
    }
    const uint64_t t0 = now_ns();
    bool on_dev = false;
    for (Job *j : b) {
      j->t_start = t0;
      running[j->ticket] = j;
      on_dev = on_dev || j->dres;
    }
    // the batch's device copies: a job is queued (under mu) only after the
    // event was recorded behind its copy, so the event's last record covers
    // the copies of every queued job
    bool wait_copies = false;
    if (on_dev && hipStreamWaitEvent(stream, copy_ev, 0) != hipSuccess) {
      (void)hipGetLastError();
      wait_copies = true;
    }
    lk.unlock();
    if (wait_copies) (void)hipStreamSynchronize(copy_stream);
    std::vector<kd_status> st(b.size(), KD_OK);
    run_batch(b, st);
    const uint64_t t1 = now_ns();
    lk.lock();
    for (uint32_t q = 0; q < b.size(); q++) {
      running.erase(b[q]->ticket);
      finish_locked(b[q], st[q], (uint32_t)b.size(), t1);
    }
    admit_locked();
    cv_done.notify_all();
  }
}

extern "C" kd_status kd_server_create(int device, const kd_server_opts *opts, kd_server **out) {
  if (!opts || !out) return KD_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return KD_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return KD_EDEVICE;
  kd_server *s = new (std::nothrow) kd_server;
  if (!s) return KD_ENOMEM;
  s->device = device;
  s->opts = *opts;
  s->arena.mirrored = opts->no_mirror == 0;
  for (uint64_t b = 0; b < opts->host_arena_bytes; b += Arena::kChunk)
    if (!s->arena.add_chunk(true)) break;  // fewer up front: more chunks are taken as jobs need them
  if (opts->host_arena_bytes) {
    // the batch buffers, sized for a batch whose residues fill the arena
    // (max_batch_seqs sequences, else a mean length of 128) and the host
    // ones written once: a batch then pays neither their allocation nor
    // their first touch (they still grow when a batch needs more)
    const uint64_t nres = opts->host_arena_bytes;
    const uint64_t n = opts->max_batch_seqs ? opts->max_batch_seqs : std::max<uint64_t>(nres / 128, 1);
    const uint64_t outb = 24 * n;  // ranks, bucket, order and at most 2 n bucket offsets
    const uint64_t head = 8 * (n + 1) + 16 + sizeof(Piece) * (nres / kPiece + 4096);  // 4,096 jobs
    if (s->h_in.reserve(head) == hipSuccess) std::memset(s->h_in.p, 0, s->h_in.cap);
    if (s->h_out.reserve(outb) == hipSuccess) std::memset(s->h_out.p, 0, s->h_out.cap);
    (void)s->d_in.reserve(head + nres);
    (void)s->d_out.reserve(outb + 256);
  }
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return KD_EDEVICE;
  }
  if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->copy_ev, hipEventDisableTiming) != hipSuccess) {
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return KD_EDEVICE;
  }
  kd_status rc = kd_ctx_create(device, s->stream, &s->ctx);
  if (rc != KD_OK) {
    (void)hipEventDestroy(s->copy_ev);
    (void)hipStreamDestroy(s->copy_stream);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return rc;
  }
  try {
    s->worker = std::thread([s] { s->loop(); });
  } catch (...) {
    kd_ctx_destroy(s->ctx);
    (void)hipEventDestroy(s->copy_ev);
    (void)hipStreamDestroy(s->copy_stream);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return KD_ENOMEM;
  }
  *out = s;
  return KD_OK;
}

extern "C" kd_status kd_server_submit(kd_server *s, const kd_job *job, uint64_t *ticket) {
  if (!s || !job || !ticket) return KD_EINVAL;
  const uint32_t N = job->n_seqs;
  if (N == 0 || !job->offsets || !job->residues || job->B == 0 || job->B > N ||
      job->B > kd::kMaxBuckets || !(job->delta > 0.0) || !std::isfinite(job->delta))
    return KD_EINVAL;
  if (job->offsets[0] != 0 || job->offsets[N] != job->n_residues) return KD_EINVAL;
  for (uint32_t i = 0; i < N; i++)
    if (job->offsets[i + 1] < job->offsets[i]) return KD_EINVAL;
  const uint64_t bytes = KD_JOB_BYTES(job->n_residues, N);
  if (bytes > s->opts.hbm_budget) return KD_EBUSY;
  Job *j = new (std::nothrow) Job;
  if (!j) return KD_ENOMEM;
  DeviceScope dev(s->device);  // a new chunk's mirror, the copy to it
  {
    std::lock_guard<std::mutex> g(s->mu);
    j->chunk = s->arena.alloc(job->n_residues, j->res);
    if (j->chunk >= 0) j->dres = s->arena.mirror(j->chunk, j->res);
  }
  try {
    if (j->chunk < 0) {
      j->own.assign(job->residues, job->residues + job->n_residues);
      j->res = j->own.data();
    } else {
      std::memcpy(j->res, job->residues, job->n_residues);
    }
    j->offsets.assign(job->offsets, job->offsets + N + 1);
  } catch (...) {
    std::lock_guard<std::mutex> g(s->mu);
    s->arena.release(j->chunk);
    delete j;
    return KD_ENOMEM;
  }
  // the residues start for the device now, overlapping running batches
  if (j->dres && hipMemcpyAsync(const_cast<uint8_t *>(j->dres), j->res, job->n_residues, hipMemcpyHostToDevice,
                                s->copy_stream) != hipSuccess) {
    (void)hipGetLastError();
    j->dres = nullptr;  // the batch sends them from the host copy
  }
  j->out = *job;
  j->out.residues = nullptr;
  j->out.offsets = nullptr;
  j->bytes = bytes;
  j->t_submit = now_ns();
  std::lock_guard<std::mutex> g(s->mu);
  if (j->dres && hipEventRecord(s->copy_ev, s->copy_stream) != hipSuccess) {
    (void)hipGetLastError();
    j->dres = nullptr;
  }
  j->ticket = s->next_ticket++;
  *ticket = j->ticket;
  s->waiting.push_back(j);
  s->admit_locked();
  s->cv_work.notify_one();
  return KD_OK;
}

extern "C" kd_status kd_server_poll(kd_server *s, kd_done *out, uint32_t max, uint32_t *n,
                                    int64_t wait_ns) {
  if (!s || !n || (max && !out)) return KD_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ns > 0)
    s->cv_done.wait_for(lk, std::chrono::nanoseconds(wait_ns), [&] { return !s->done.empty(); });
  uint32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return KD_OK;
}

extern "C" kd_status kd_server_cancel(kd_server *s, uint64_t ticket) {
  if (!s) return KD_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->running.count(ticket)) return KD_EBUSY;
  for (auto *q : {&s->waiting, &s->admitted}) {
    for (auto it = q->begin(); it != q->end(); ++it) {
      if ((*it)->ticket != ticket) continue;
      Job *j = *it;
      const bool was_admitted = q == &s->admitted;
      q->erase(it);
      if (!was_admitted) s->reserved += j->bytes;  // finish_locked releases the charge
      s->finish_locked(j, KD_ECANCELLED, 0, now_ns());
      s->admit_locked();  // the freed budget may admit waiting jobs
      s->cv_work.notify_one();
      s->cv_done.notify_all();
      return KD_OK;
    }
  }
  return KD_EINVAL;
}

extern "C" kd_status kd_server_status(kd_server *s, uint32_t *waiting, uint32_t *admitted,
                                      uint32_t *running, uint32_t *done, uint64_t *reserved) {
  if (!s) return KD_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (waiting) *waiting = (uint32_t)s->waiting.size();
  if (admitted) *admitted = (uint32_t)s->admitted.size();
  if (running) *running = (uint32_t)s->running.size();
  if (done) *done = (uint32_t)s->done.size();
  if (reserved) *reserved = s->reserved;
  return KD_OK;
}

extern "C" void kd_server_destroy(kd_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Job *j : s->waiting) delete j;
  for (Job *j : s->admitted) delete j;
  (void)hipSetDevice(s->device);
  kd_ctx_destroy(s->ctx);  // synchronizes the stream
  (void)hipStreamSynchronize(s->copy_stream);  // copies of jobs that never ran
  if (s->d_in.p) (void)hipFree(s->d_in.p);
  if (s->d_out.p) (void)hipFree(s->d_out.p);
  s->d_in.p = s->d_out.p = nullptr;
  (void)hipEventDestroy(s->copy_ev);
  (void)hipStreamDestroy(s->copy_stream);
  (void)hipStreamDestroy(s->stream);
  delete s;  // the arena: pinned chunks and their device mirrors
}
