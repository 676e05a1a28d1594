// Request server (kd_server_*): admission against a device-memory budget
// and continuous batching of independent jobs onto the batched path.
//
// Jobs move  waiting --(fits the budget)--> admitted --(picked by a batch)-->
// running --> done (a completion record waits for kd_server_poll).
//
// One worker thread runs batches through two stages on two streams of the
// same (default) priority, each with a context of its own:
//   stage A (count stream): gather the batch's input, count and lay out
//            every set (kmer_count_batch, which synchronizes stream A once);
//   stage B (rank stream):  rank and split every set, copy the results back.
// While batch k is in stage B, the worker already takes the jobs that
// arrived meanwhile as batch k+1 and runs its stage A, so the counting of
// arriving jobs overlaps the rank launch of the running batch on the device
// and the host work (gather tables, layout sizing, work lists) overlaps both.
// Batch k's results are written, and batch k+1's stage B enqueued (behind
// an event on stream A), once batch k's stage B has completed.  A job with
// bad input fails alone: its batch is counted again without it.  A job's
// residues go to the device when it is submitted (a copy stream of their
// own), so a batch finds its input there and only gathers it into one
// buffer.
#include <time.h>

#include <algorithm>
#include <chrono>
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
  bool mirrored = true;       // chunks get device mirrors ...
  uint64_t mirror_limit = 0;  // ... while their bytes stay within this
  uint64_t mirror_bytes = 0;  // device bytes held by mirrors (charged to the budget)
  bool add_chunk(bool touch) {
    void *v = nullptr;
    if (hipHostMalloc(&v, kChunk, hipHostMallocNonCoherent) != hipSuccess) return false;
    uint8_t *p = static_cast<uint8_t *>(v);
    if (touch) std::memset(p, 0, kChunk);
    void *d = nullptr;
    if (mirrored && mirror_bytes + kChunk <= mirror_limit) {
      if (hipMalloc(&d, kChunk) != hipSuccess) {
        (void)hipGetLastError();
        d = nullptr;
      } else {
        mirror_bytes += kChunk;
      }
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

// A batch between its two stages: counted on stream A, ranked on stream B.
struct Flight {
  std::vector<Job *> b;            // the batch's jobs
  std::vector<kd_status> st;       // per job; KD_OK while it is live
  std::vector<uint32_t> live;      // indices into b of the jobs in the counted set
  std::vector<uint32_t> first, Bs;
  uint32_t N = 0;
  uint64_t nb = 0;                 // bucket offsets of all sets
  kd_set *set = nullptr;           // counted on ctx_a
  hipEvent_t ev[4] = {};           // timeline: count start/end (A), rank start/end (B)
  hipEvent_t done_ev = nullptr;    // stage B complete
  bool timed = false;
};

struct kd_server {
  int device = 0;
  kd_server_opts opts{};
  hipStream_t stream = nullptr;       // stage B: rank, split, results back
  hipStream_t stream_a = nullptr;     // stage A: gather, count, layout
  hipStream_t copy_stream = nullptr;  // the jobs' copies at submit
  hipEvent_t copy_ev = nullptr;       // recorded after each of them (under mu)
  hipEvent_t counted_ev = nullptr;    // stage A of the next batch done (stream A)
  hipEvent_t base_ev = nullptr;       // timeline origin (stream A, at creation)
  kd_ctx *ctx = nullptr;              // stage B
  kd_ctx *ctx_a = nullptr;            // stage A
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<Job *> waiting, admitted;
  std::unordered_map<uint64_t, Job *> running;
  std::deque<kd_done> done;
  uint64_t reserved = 0;  // charges of the admitted and running jobs
  Arena arena;  // the jobs' residues (pinned) and their device mirrors
  // staging, used by the worker only: inputs (stage A), outputs (stage B)
  HostBuf h_in, h_out;
  DevBuf d_in, d_out;
  // timeline (opts.timeline): device milliseconds since base_ev of each
  // batch's stages, guarded by mu
  std::vector<kd_server_stage> stages;

  void admit_locked() {  // FIFO: the oldest waiting job goes first
    while (!waiting.empty() &&
           reserved + arena.mirror_bytes + waiting.front()->bytes <= opts.hbm_budget) {
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

  void release_streams() {
    for (hipEvent_t e : {copy_ev, counted_ev, base_ev})
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t t : {copy_stream, stream_a, stream})
      if (t) (void)hipStreamDestroy(t);
  }
  kd_status count_stage(Flight &f);
  kd_status rank_stage(Flight &f);
  void results(Flight &f);
  void loop();
};

// Stage A of a batch (every st[q] KD_OK on entry): its input gathered and
// every set counted and laid out on stream A (ctx_a).  A job with bad input
// is marked and the batch counted again without it.  On return f.set holds
// the live jobs' sets (null when none is left or on a device error, with
// st[] set accordingly).
kd_status kd_server::count_stage(Flight &f) {
  std::vector<Job *> &b = f.b;
  std::vector<kd_status> &st = f.st;
  for (;;) {
    f.live.clear();
    for (uint32_t q = 0; q < b.size(); q++)
      if (st[q] == KD_OK) f.live.push_back(q);
    if (f.live.empty()) return KD_OK;
    const uint32_t ns = (uint32_t)f.live.size();
    f.first.assign(ns + 1, 0);
    f.Bs.assign(ns, 0);
    uint64_t nres = 0;
    for (uint32_t k = 0; k < ns; k++) {
      const Job *j = b[f.live[k]];
      f.first[k + 1] = f.first[k] + j->out.n_seqs;
      f.Bs[k] = j->out.B;
      nres += j->out.n_residues;
    }
    const uint32_t N = f.first[ns];
    f.N = N;
    uint64_t npc = 0;
    f.nb = 0;
    for (uint32_t k = 0; k < ns; k++) {
      f.nb += f.Bs[k] + 1;
      const Job *j = b[f.live[k]];
      if (j->dres) npc += (j->out.n_residues + kPiece - 1) / kPiece;
    }
    // input: offsets (N+1 u64, rebased) and the gather pieces, staged in
    // pinned memory, then the residues (gathered from the jobs' device
    // copies; a job without one is sent from its host copy)
    const size_t tab_at = (8ull * (N + 1) + 15) & ~(size_t)15;
    const size_t head = tab_at + sizeof(Piece) * npc;
    const size_t in_bytes = head + nres;
    if (h_in.reserve(head) != hipSuccess || d_in.reserve(in_bytes) != hipSuccess) {
      for (uint32_t q : f.live) st[q] = KD_ENOMEM;
      return KD_ENOMEM;
    }
    uint64_t *off = static_cast<uint64_t *>(h_in.p);
    Piece *pcs = reinterpret_cast<Piece *>(static_cast<char *>(h_in.p) + tab_at);
    uint8_t *d_resw = static_cast<uint8_t *>(d_in.p) + head;
    uint64_t r0 = 0, pq = 0;
    bool copied = true;
    for (uint32_t k = 0; k < ns; k++) {
      const Job *j = b[f.live[k]];
      const uint64_t n = j->out.n_residues;
      for (uint32_t i = 0; i < j->out.n_seqs; i++) off[f.first[k] + i] = r0 + j->offsets[i];
      if (j->dres) {
        for (uint64_t a = 0; a < n; a += kPiece) pcs[pq++] = Piece{j->dres + a, r0 + a, std::min(kPiece, n - a)};
      } else {
        copied = copied && hipMemcpyAsync(d_resw + r0, j->res, n, hipMemcpyHostToDevice, stream_a) == hipSuccess;
      }
      r0 += n;
    }
    off[N] = r0;
    const uint64_t *d_off = static_cast<const uint64_t *>(d_in.p);
    copied = copied && hipMemcpyAsync(d_in.p, h_in.p, head, hipMemcpyHostToDevice, stream_a) == hipSuccess;
    if (copied && npc) {
      hipLaunchKernelGGL(gather_pieces_kernel, dim3((uint32_t)npc), dim3(256), 0, stream_a,
                         reinterpret_cast<const Piece *>(static_cast<char *>(d_in.p) + tab_at), d_resw);
      copied = hipGetLastError() == hipSuccess;
    }
    if (!copied) {
      for (uint32_t x : f.live) st[x] = KD_EDEVICE;
      return KD_EDEVICE;
    }
    // the jobs' device copies and the input are read by stream A only, and
    // the next batch's input is written only after this count's own
    // synchronization of stream A
    kd_status rc = kmer_count_batch(ctx_a, d_resw, d_off, nres, ns, f.first.data(), &f.set);
    if (rc == KD_EBADRESIDUE || rc == KD_ESHORTSEQ || rc == KD_ETOOLONG) {
      // the job holding the offending sequence fails; the others are counted again
      uint64_t seq = 0, pos = 0;
      kd_last_error_info(ctx_a, &seq, &pos);
      const uint32_t k =
          (uint32_t)(std::upper_bound(f.first.begin(), f.first.end(), (uint32_t)seq) - f.first.begin()) - 1;
      st[f.live[std::min(k, ns - 1)]] = rc;
      f.set = nullptr;
      continue;
    }
    if (rc != KD_OK) {
      for (uint32_t q : f.live) st[q] = rc;
      f.set = nullptr;
    }
    return rc;
  }
}

// Stage B, enqueued on stream B behind stage A's completion: rank and split
// of every set, results to the pinned host buffer, then the batch's done
// event.  The set was counted on ctx_a; it is ranked on ctx (its blocks stay
// with ctx_a's pool, which gets them back when the set is destroyed after
// stage B has completed).
kd_status kd_server::rank_stage(Flight &f) {
  if (!f.done_ev) {
    for (uint32_t q : f.live) f.st[q] = KD_EDEVICE;
    return KD_EDEVICE;
  }
  const uint32_t N = f.N, ns = (uint32_t)f.live.size();
  const size_t out_bytes = 8ull * N + 4ull * N + 4ull * N + 4ull * f.nb;
  kd_status rc = KD_OK;
  if (h_out.reserve(out_bytes) != hipSuccess || d_out.reserve(out_bytes + 256) != hipSuccess) rc = KD_ENOMEM;
  if (rc == KD_OK && (hipEventRecord(counted_ev, stream_a) != hipSuccess ||
                      hipStreamWaitEvent(stream, counted_ev, 0) != hipSuccess))
    rc = KD_EDEVICE;
  if (rc == KD_OK && f.timed && hipEventRecord(f.ev[2], stream) != hipSuccess) rc = KD_EDEVICE;
  char *dout = static_cast<char *>(d_out.p);
  double *d_ranks = reinterpret_cast<double *>(dout);
  uint32_t *d_bucket = reinterpret_cast<uint32_t *>(dout + 8ull * N);
  uint32_t *d_order = d_bucket + N;
  uint32_t *d_offs = d_order + N;
  f.set->ctx = ctx;
  if (rc == KD_OK) rc = kmer_rank(ctx, f.set, f.b[f.live[0]]->out.delta, d_ranks);
  if (rc == KD_OK)
    rc = sample_partition_batch(ctx, d_ranks, ns, f.first.data(), f.Bs.data(), d_bucket, d_order, d_offs,
                                nullptr, nullptr);
  f.set->ctx = ctx_a;
  if (rc == KD_OK && hipMemcpyAsync(h_out.p, d_out.p, out_bytes, hipMemcpyDeviceToHost, stream) != hipSuccess)
    rc = KD_EDEVICE;
  if (rc == KD_OK && f.timed && hipEventRecord(f.ev[3], stream) != hipSuccess) rc = KD_EDEVICE;
  if (rc == KD_OK && hipEventRecord(f.done_ev, stream) != hipSuccess) rc = KD_EDEVICE;
  if (rc != KD_OK)
    for (uint32_t q : f.live) f.st[q] = rc;
  return rc;
}

// After stage B: waits for it, writes the live jobs' results into their
// buffers and releases the set.
void kd_server::results(Flight &f) {
  const bool ok = hipStreamSynchronize(stream) == hipSuccess;
  if (f.set) {
    kd_set_destroy(f.set);
    f.set = nullptr;
  }
  if (!ok) {
    for (uint32_t q : f.live) f.st[q] = KD_EDEVICE;
    return;
  }
  const uint32_t N = f.N;
  const char *hout = static_cast<const char *>(h_out.p);
  const double *h_ranks = reinterpret_cast<const double *>(hout);
  const uint32_t *h_bucket = reinterpret_cast<const uint32_t *>(hout + 8ull * N);
  const uint32_t *h_order = h_bucket + N;
  const uint32_t *h_offs = h_order + N;
  uint64_t ob = 0;
  for (uint32_t k = 0; k < f.live.size(); k++) {
    if (f.st[f.live[k]] != KD_OK) continue;
    const kd_job &o = f.b[f.live[k]]->out;
    const uint32_t a = f.first[k], n = o.n_seqs;
    if (o.ranks) std::memcpy(o.ranks, h_ranks + a, 8ull * n);
    if (o.bucket) std::memcpy(o.bucket, h_bucket + a, 4ull * n);
    if (o.order) std::memcpy(o.order, h_order + a, 4ull * n);
    if (o.bucket_offsets) std::memcpy(o.bucket_offsets, h_offs + ob, 4ull * (o.B + 1));
    ob += o.B + 1;
  }
  if (f.timed) {
    kd_server_stage t{};
    float ms[4] = {0.f, 0.f, 0.f, 0.f};
    bool good = true;
    for (int i = 0; i < 4; i++) good = good && hipEventElapsedTime(&ms[i], base_ev, f.ev[i]) == hipSuccess;
    if (good) {
      t.count_start_ms = ms[0];
      t.count_end_ms = ms[1];
      t.rank_start_ms = ms[2];
      t.rank_end_ms = ms[3];
      t.jobs = (uint32_t)f.b.size();
      std::lock_guard<std::mutex> g(mu);
      stages.push_back(t);
    } else {
      (void)hipGetLastError();
    }
  }
}

void kd_server::loop() {
  (void)hipSetDevice(device);
  Flight fl[2];
  for (Flight &f : fl) {
    for (hipEvent_t &e : f.ev)
      if (opts.timeline && hipEventCreate(&e) != hipSuccess) e = nullptr;
    if (hipEventCreateWithFlags(&f.done_ev, hipEventDisableTiming) != hipSuccess) f.done_ev = nullptr;
  }
  Flight *busy = nullptr;  // the batch in stage B
  int next = 0;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || !admitted.empty() || busy; });
    // while a batch is in stage B, jobs arriving before it completes start
    // their stage A at once (short waits, the event polled in between)
    while (busy && !stop && admitted.empty() && hipEventQuery(busy->done_ev) == hipErrorNotReady)
      cv_work.wait_for(lk, std::chrono::microseconds(50), [&] { return stop || !admitted.empty(); });
    if (stop && !busy) break;
    Flight *f = nullptr;
    if (!stop && !admitted.empty()) {
      // the batch: admitted jobs of the oldest job's delta, in FIFO order
      f = &fl[next];
      next ^= 1;
      f->b.clear();
      const double delta = admitted.front()->out.delta;
      uint64_t seqs = 0;
      for (auto it = admitted.begin(); it != admitted.end();) {
        Job *j = *it;
        if (opts.max_batch_jobs && f->b.size() >= opts.max_batch_jobs) break;
        if (j->out.delta != delta) {
          ++it;
          continue;
        }
        if (!f->b.empty() && opts.max_batch_seqs && seqs + j->out.n_seqs > opts.max_batch_seqs) break;
        seqs += j->out.n_seqs;
        f->b.push_back(j);
        it = admitted.erase(it);
      }
      const uint64_t t0 = now_ns();
      bool on_dev = false;
      for (Job *j : f->b) {
        j->t_start = t0;
        running[j->ticket] = j;
        on_dev = on_dev || j->dres;
      }
      // the batch's device copies: a job is queued (under mu) only after the
      // event was recorded behind its copy, so the event's last record covers
      // the copies of every queued job
      bool wait_copies = false;
      if (on_dev && hipStreamWaitEvent(stream_a, copy_ev, 0) != hipSuccess) {
        (void)hipGetLastError();
        wait_copies = true;
      }
      lk.unlock();
      if (wait_copies) (void)hipStreamSynchronize(copy_stream);
      f->st.assign(f->b.size(), KD_OK);
      f->timed = opts.timeline && f->ev[0] && f->ev[1] && f->ev[2] && f->ev[3];
      if (f->timed && hipEventRecord(f->ev[0], stream_a) != hipSuccess) f->timed = false;
      count_stage(*f);  // overlaps the running batch's stage B
      if (f->timed && hipEventRecord(f->ev[1], stream_a) != hipSuccess) f->timed = false;
    } else {
      lk.unlock();
    }
    // the running batch: results out, jobs done
    if (busy) {
      results(*busy);
      const uint64_t t1 = now_ns();
      lk.lock();
      for (uint32_t q = 0; q < busy->b.size(); q++) {
        running.erase(busy->b[q]->ticket);
        finish_locked(busy->b[q], busy->st[q], (uint32_t)busy->b.size(), t1);
      }
      admit_locked();
      cv_done.notify_all();
      lk.unlock();
      busy = nullptr;
    }
    // the new batch's stage B (or, with nothing to rank, its jobs are done)
    if (f) {
      if (f->set && rank_stage(*f) == KD_OK) {
        busy = f;
      } else {
        if (f->set) results(*f);
        const uint64_t t1 = now_ns();
        lk.lock();
        for (uint32_t q = 0; q < f->b.size(); q++) {
          running.erase(f->b[q]->ticket);
          finish_locked(f->b[q], f->st[q], (uint32_t)f->b.size(), t1);
        }
        admit_locked();
        cv_done.notify_all();
        lk.unlock();
      }
    }
    lk.lock();
  }
  lk.unlock();
  for (Flight &f : fl) {
    for (hipEvent_t e : f.ev)
      if (e) (void)hipEventDestroy(e);
    if (f.done_ev) (void)hipEventDestroy(f.done_ev);
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
  s->arena.mirror_limit = opts->hbm_budget / 2;  // the rest of the budget stays for jobs
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
      hipStreamCreateWithFlags(&s->stream_a, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->copy_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->counted_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&s->base_ev) != hipSuccess || hipEventRecord(s->base_ev, s->stream_a) != hipSuccess) {
    s->release_streams();
    delete s;
    return KD_EDEVICE;
  }
  kd_status rc = kd_ctx_create(device, s->stream, &s->ctx);
  if (rc == KD_OK) rc = kd_ctx_create(device, s->stream_a, &s->ctx_a);
  if (rc != KD_OK) {
    if (s->ctx) kd_ctx_destroy(s->ctx);
    s->release_streams();
    delete s;
    return rc;
  }
  try {
    s->worker = std::thread([s] { s->loop(); });
  } catch (...) {
    kd_ctx_destroy(s->ctx);
    kd_ctx_destroy(s->ctx_a);
    s->release_streams();
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
  if (reserved) *reserved = s->reserved + s->arena.mirror_bytes;
  return KD_OK;
}

extern "C" kd_status kd_server_timeline(kd_server *s, kd_server_stage *out, uint32_t max, uint32_t *n) {
  if (!s || !n || (max && !out)) return KD_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  const uint32_t k = (uint32_t)std::min<size_t>(max, s->stages.size());
  for (uint32_t i = 0; i < k; i++) out[i] = s->stages[i];
  s->stages.erase(s->stages.begin(), s->stages.begin() + k);
  *n = k;
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
  kd_ctx_destroy(s->ctx);    // synchronizes stream B
  kd_ctx_destroy(s->ctx_a);  // synchronizes stream A
  (void)hipStreamSynchronize(s->copy_stream);  // copies of jobs that never ran
  if (s->d_in.p) (void)hipFree(s->d_in.p);
  if (s->d_out.p) (void)hipFree(s->d_out.p);
  s->d_in.p = s->d_out.p = nullptr;
  s->release_streams();
  delete s;  // the arena: pinned chunks and their device mirrors
}
