"""MI355X (gfx950) k-mer rank + regular-sampling decomposition.

Thin ctypes binding over ``libkmerdecomp.so`` (declared in ``include/kd.h``).
Every step runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch provides device memory and the stream: tensors passed in
must live on the context's GPU, and results come back as CUDA tensors.

    import paper_0905_1744_amd as kd
    ctx = kd.Context()                       # on torch's current stream
    kset = ctx.kmer_count(residues, offsets) # uint8 / int64 CUDA tensors
    ranks = ctx.kmer_rank(kset, delta=0.1)   # float64 [N]
    part = ctx.sample_partition(ranks, B=16) # bucket / order / offsets ...

There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # must load before the library so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmerdecomp.so")
_lib = None

KD_OK = 0
STATUS = {0: "KD_OK", -1: "KD_EINVAL", -2: "KD_EBADRESIDUE", -3: "KD_ESHORTSEQ",
          -4: "KD_ETOOLONG", -5: "KD_ENOMEM", -6: "KD_EBUSY", -7: "KD_EDEVICE",
          -8: "KD_ECANCELLED", -9: "KD_ETOOLARGE"}
WORDS = 46656


class KdError(RuntimeError):
    def __init__(self, status: int, what: str, seq=None, pos=None):
        msg = f"{what}: {STATUS.get(status, status)} ({lib().kd_strerror(status).decode()})"
        if seq is not None:
            msg += f" at sequence {seq}, position {pos}"
        super().__init__(msg)
        self.status, self.seq, self.pos = status, seq, pos


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_batch_jobs", C.c_uint32), ("max_batch_seqs", C.c_uint32),
                ("host_arena_bytes", C.c_uint64), ("no_mirror", C.c_uint32), ("timeline", C.c_uint32)]


class ServerStage(C.Structure):
    _fields_ = [("count_start_ms", C.c_double), ("count_end_ms", C.c_double), ("rank_start_ms", C.c_double),
                ("rank_end_ms", C.c_double), ("jobs", C.c_uint32), ("reserved0", C.c_uint32)]


class Job(C.Structure):
    _fields_ = [("residues", C.c_void_p), ("offsets", C.c_void_p), ("n_seqs", C.c_uint32),
                ("n_residues", C.c_uint64), ("B", C.c_uint32), ("delta", C.c_double),
                ("ranks", C.c_void_p), ("bucket", C.c_void_p), ("order", C.c_void_p),
                ("bucket_offsets", C.c_void_p)]


class Done(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("batch_jobs", C.c_uint32),
                ("t_submit_ns", C.c_uint64), ("t_start_ns", C.c_uint64), ("t_done_ns", C.c_uint64)]


def job_bytes(n_residues: int, n_seqs: int) -> int:
    """Device bytes the server charges a job against its budget (KD_JOB_BYTES)."""
    return 8 * n_residues + 256 * n_seqs + 65536


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_0905_1744_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    P, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32
    PP = C.POINTER(C.c_void_p)
    sig = {
        "kd_ctx_create": (i32, [C.c_int, P, PP]),
        "kd_ctx_destroy": (None, [P]),
        "kd_strerror": (C.c_char_p, [i32]),
        "kd_last_error_info": (i32, [P, C.POINTER(u64), C.POINTER(u64)]),
        "kd_ctx_synchronize": (i32, [P]),
        "kd_ctx_stream": (P, [P]),
        "kd_ctx_enable_timing": (i32, [P, C.c_int]),
        "kd_ctx_stage_time": (i32, [P, C.c_int, C.POINTER(C.c_double), C.POINTER(u64)]),
        "kd_ctx_reset_timing": (i32, [P]),
        "kmer_count": (i32, [P, P, P, u32, u64, PP]),
        "kd_set_size": (u32, [P]),
        "kd_set_entries": (u64, [P]),
        "kd_set_export_lists": (i32, [P, P, P, P, P]),
        "kd_set_export_dense": (i32, [P, P, u32, u32, P]),
        "kd_set_destroy": (None, [P]),
        "kmer_similarity": (i32, [P, P, u32, u32, u32, u32, P, P]),
        "kmer_rank": (i32, [P, P, C.c_double, P]),
        "sample_partition": (i32, [P, P, u32, u32, P, P, P, P, P]),
        "sample_partition_noalloc": (i32, [P, P, u32, u32, P, P, P, P, P]),
        "kmer_count_batch": (i32, [P, P, P, u64, u32, P, PP]),
        "kmer_count_blocks": (i32, [P, P, P, u32, u64, u32, PP]),
        "kd_set_count": (u32, [P]),
        "kd_set_first": (i32, [P, P]),
        "sample_partition_batch": (i32, [P, P, u32, P, P, P, P, P, P, P]),
        "kd_batch_run": (i32, [P, P, P, u64, u32, P, P, C.c_double, P, P, P, P]),
        "kd_autotune": (i32, [P, P, C.c_double, C.POINTER(u32), C.POINTER(C.c_double)]),
        "kd_ctx_set_tasks_per_cu": (i32, [P, u32, u32, u32]),
        "kmer_rank_global": (i32, [P, P, P, u32, C.c_double, P, P]),
        "kd_gather_sequences": (i32, [P, P, P, u32, u64, P, u32, P, u64, P]),
        "kmer_distance_matrices": (i32, [P, P, C.c_double, P]),
        "upgma_trees": (i32, [P, u32, P, P, P, P]),
        "psp_profile": (i32, [P, P, u32, u32, P]),
        "kd_decompose": (i32, [P, P, P, u32, u64, u32, C.c_int, C.c_double, P, P, P, P]),
        "psp_scores": (i32, [P, P, u32, P]),
        "kd_calibrate_lds": (i32, [P, u32, u32, u32, C.POINTER(C.c_double), C.POINTER(u64)]),
        "kd_batch_plan_create": (i32, [P, P, P, u64, u32, P, P, C.c_double, P, P, P, P, PP]),
        "kd_batch_plan_launch": (i32, [P]),
        "kd_batch_plan_launches": (u32, [P]),
        "kd_batch_plan_destroy": (None, [P]),
        "kd_server_create": (i32, [C.c_int, C.POINTER(ServerOpts), PP]),
        "kd_server_submit": (i32, [P, C.POINTER(Job), C.POINTER(u64)]),
        "kd_server_poll": (i32, [P, C.POINTER(Done), u32, C.POINTER(u32), C.c_int64]),
        "kd_server_cancel": (i32, [P, u64]),
        "kd_server_status": (i32, [P, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32), C.POINTER(u32),
                                   C.POINTER(u64)]),
        "kd_server_destroy": (None, [P]),
        "kd_server_timeline": (i32, [P, C.POINTER(ServerStage), u32, C.POINTER(u32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev_tensor(x, dtype, device):
    """numpy array or tensor -> contiguous CUDA tensor of the given dtype."""
    if isinstance(x, torch.Tensor):
        t = x
    else:
        a = np.ascontiguousarray(x)
        if not a.flags.writeable:  # torch.from_numpy wants writable memory (the copy is only read)
            a = a.copy()
        t = torch.from_numpy(a)
    if t.dtype != dtype:
        t = t.view(dtype) if t.element_size() == torch.empty((), dtype=dtype).element_size() else t.to(dtype)
    return t.to(device, non_blocking=False).contiguous()


class KmerSet:
    """Device-resident counted set (owned by the library)."""

    def __init__(self, ctx: "Context", handle: C.c_void_p):
        self.ctx, self.handle = ctx, handle

    @property
    def n(self) -> int:
        return int(lib().kd_set_size(self.handle))

    @property
    def nsets(self) -> int:
        return int(lib().kd_set_count(self.handle))

    @property
    def entries(self) -> int:
        return int(lib().kd_set_entries(self.handle))

    def set_first(self) -> np.ndarray:
        """Bounds of the sets it holds (nsets + 1 entries)."""
        f = np.zeros(self.nsets + 1, dtype=np.uint32)
        st = lib().kd_set_first(self.handle, f.ctypes.data_as(C.c_void_p))
        if st != KD_OK:
            raise KdError(st, "kd_set_first")
        return f

    def export_lists(self):
        """(ids u16, counts u16, off u64) as CUDA tensors (int16/int16/int64 storage)."""
        dev = self.ctx.device
        ids = torch.empty(max(self.entries, 1), dtype=torch.int16, device=dev)
        cnt = torch.empty(max(self.entries, 1), dtype=torch.int16, device=dev)
        off = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        self.ctx._check(lib().kd_set_export_lists(self.ctx.handle, self.handle, _ptr(ids), _ptr(cnt),
                                                  _ptr(off)), "kd_set_export_lists")
        return ids[:self.entries], cnt[:self.entries], off

    def export_dense(self, first: int, count: int):
        out = torch.empty((count, WORDS), dtype=torch.int16, device=self.ctx.device)
        self.ctx._check(lib().kd_set_export_dense(self.ctx.handle, self.handle, first, count, _ptr(out)),
                        "kd_set_export_dense")
        return out

    def destroy(self):
        if self.handle:
            lib().kd_set_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.destroy()
        except Exception:
            pass


class PspPair(C.Structure):
    _fields_ = [("fx", C.c_void_p), ("lx", C.c_uint32), ("ly", C.c_uint32), ("fy", C.c_void_p),
                ("scores", C.c_void_p)]


class Context:
    """A library context bound to one GPU and one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        out = C.c_void_p()
        st = L.kd_ctx_create(device, C.c_void_p(h), C.byref(out))
        if st != KD_OK:
            raise KdError(st, "kd_ctx_create")
        self.handle = out

    def _check(self, st, what):
        if st != KD_OK:
            seq = pos = None
            if st in (-2, -3, -4):
                s, p = C.c_uint64(), C.c_uint64()
                lib().kd_last_error_info(self.handle, C.byref(s), C.byref(p))
                seq, pos = int(s.value), int(p.value)
            raise KdError(st, what, seq, pos)

    def close(self):
        if getattr(self, "handle", None):
            lib().kd_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    STAGES = ("count", "layout", "pairs", "finalize", "partition", "similarity", "global", "gather",
              "dist", "tree", "psp")

    def enable_timing(self, on: bool = True, stages=None):
        """Time every stage, or only the named ones (each costs two events)."""
        arg = 0
        if on:
            arg = 1 if stages is None else 0x10000 | sum(1 << self.STAGES.index(n) for n in stages)
        self._check(lib().kd_ctx_enable_timing(self.handle, arg), "kd_ctx_enable_timing")

    def reset_timing(self):
        self._check(lib().kd_ctx_reset_timing(self.handle), "kd_ctx_reset_timing")

    def stage_times(self):
        """{stage: (total_ms, launches)} since the last reset (synchronizes)."""
        out = {}
        for i, name in enumerate(self.STAGES):
            ms, n = C.c_double(), C.c_uint64()
            self._check(lib().kd_ctx_stage_time(self.handle, i, C.byref(ms), C.byref(n)), "kd_ctx_stage_time")
            out[name] = (ms.value, int(n.value))
        return out

    def synchronize(self):
        self._check(lib().kd_ctx_synchronize(self.handle), "kd_ctx_synchronize")

    # -------------------------------------------------------------- calls
    def kmer_count(self, residues, offsets) -> KmerSet:
        res = _dev_tensor(residues, torch.uint8, self.device)
        off = _dev_tensor(offsets, torch.int64, self.device)
        n = off.numel() - 1
        out = C.c_void_p()
        self._check(lib().kmer_count(self.handle, _ptr(res), _ptr(off), n, res.numel(), C.byref(out)),
                    "kmer_count")
        return KmerSet(self, out)

    def kmer_similarity(self, kset: KmerSet, r0: int, nr: int, c0: int, nc: int, denom: bool = False):
        S = torch.empty((nr, nc), dtype=torch.int16, device=self.device)
        Dn = torch.empty((nr, nc), dtype=torch.int16, device=self.device) if denom else None
        self._check(lib().kmer_similarity(self.handle, kset.handle, r0, nr, c0, nc, _ptr(S), _ptr(Dn)),
                    "kmer_similarity")
        return (S, Dn) if denom else S

    TUNE_SHAPES = (8, 16, 32, 64, 128)

    def autotune(self, kset: KmerSet, delta: float = 0.1):
        """Pick the rank kernel's work-list shape for sets of this size class
        (kd_autotune); returns (tasks per compute unit, {shape: ms})."""
        best = C.c_uint32()
        ms = (C.c_double * len(self.TUNE_SHAPES))()
        self._check(lib().kd_autotune(self.handle, kset.handle, float(delta), C.byref(best), ms), "kd_autotune")
        return int(best.value), dict(zip(self.TUNE_SHAPES, list(ms)))

    def set_tasks_per_cu(self, nsets: int, n: int, tasks: int):
        self._check(lib().kd_ctx_set_tasks_per_cu(self.handle, nsets, n, tasks), "kd_ctx_set_tasks_per_cu")

    def kmer_rank(self, kset: KmerSet, delta: float = 0.1, out=None):
        R = out if out is not None else torch.empty(kset.n, dtype=torch.float64, device=self.device)
        self._check(lib().kmer_rank(self.handle, kset.handle, float(delta), _ptr(R)), "kmer_rank")
        return R

    def sample_partition(self, ranks, B: int):
        R = _dev_tensor(ranks, torch.float64, self.device)
        n = R.numel()
        bucket = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        order = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        offsets = torch.empty(B + 1 if B > 0 else 1, dtype=torch.int32, device=self.device)
        pr = torch.empty(max(B - 1, 1), dtype=torch.float64, device=self.device)
        pi = torch.empty(max(B - 1, 1), dtype=torch.int32, device=self.device)
        self._check(lib().sample_partition(self.handle, _ptr(R), n, B, _ptr(bucket), _ptr(order),
                                           _ptr(offsets), _ptr(pr), _ptr(pi)), "sample_partition")
        return dict(bucket=bucket[:n], order=order[:n], offsets=offsets, pivot_rank=pr[:max(B - 1, 0)],
                    pivot_idx=pi[:max(B - 1, 0)])

    def sample_partition_noalloc(self, ranks, B: int, out):
        """sample_partition through the entry point that allocates no device
        memory.  `ranks` is a device f64 tensor and `out` a dict of
        preallocated device tensors (bucket, order: int32[n]; offsets:
        int32[B+1]; pivot_rank f64[B-1] and pivot_idx int32[B-1], each may be
        None) which receive the results."""
        n = ranks.numel()
        self._check(lib().sample_partition_noalloc(
            self.handle, _ptr(ranks), n, B, _ptr(out["bucket"]), _ptr(out["order"]),
            _ptr(out["offsets"]), _ptr(out.get("pivot_rank")), _ptr(out.get("pivot_idx"))),
            "sample_partition_noalloc")
        return out

    def calibrate_lds(self, workgroups: int, steps: int, batch: int):
        """(milliseconds, 64-lane LDS reads) of the random-read probe."""
        ms, n = C.c_double(), C.c_uint64()
        self._check(lib().kd_calibrate_lds(self.handle, workgroups, steps, batch, C.byref(ms),
                                           C.byref(n)), "kd_calibrate_lds")
        return float(ms.value), int(n.value)

    # ---------------------------------------------------- globalized rank
    def kmer_rank_global(self, blocks: KmerSet, local_ranks, k: int, delta: float = 0.1, out=None):
        """Globalized rank (Section 3.1.1; Algorithm 2 steps 3-6) of a set
        counted block by block; local_ranks = kmer_rank(blocks).  Returns
        (ranks, samples): samples are the k * nsets input indices picked."""
        loc = _dev_tensor(local_ranks, torch.float64, self.device)
        if loc.numel() != blocks.n:
            raise ValueError(f"local_ranks: expected {blocks.n} entries, got {loc.numel()}")
        R = out if out is not None else torch.empty(blocks.n, dtype=torch.float64, device=self.device)
        smp = torch.empty(max(int(k) * blocks.nsets, 1), dtype=torch.int32, device=self.device)
        self._check(lib().kmer_rank_global(self.handle, blocks.handle, _ptr(loc), int(k), float(delta),
                                           _ptr(R), _ptr(smp)), "kmer_rank_global")
        return R, smp[:int(k) * blocks.nsets]

    def globalized_rank(self, residues, offsets, B: int, k: int = None, delta: float = 0.1):
        """Algorithm 2 steps 1-6 on one device: count the B blocks, rank each
        against itself (local ranks), then every sequence against k samples
        per block (k defaults to B - 1).  Returns dict(local, ranks, samples)."""
        off = _dev_tensor(offsets, torch.int64, self.device)
        n = off.numel() - 1
        if not 1 <= B <= n:
            raise ValueError("need 1 <= B <= number of sequences")
        k = max(B - 1, 1) if k is None else int(k)
        kb = self.kmer_count_blocks(residues, off, B)
        try:
            loc = self.kmer_rank(kb, delta)
            R, smp = self.kmer_rank_global(kb, loc, k, delta)
        finally:
            kb.destroy()
        return dict(local=loc, ranks=R, samples=smp)

    # ---------------------------------------------------------- decompose
    def decompose(self, residues, offsets, B: int, globalized: bool = False, delta: float = 0.1):
        """Algorithm 2's front end in one call: ranks (centralized, or
        globalized with k = B - 1 samples per block) and the split into B
        buckets.  Returns dict(ranks, bucket, order, offsets)."""
        res = _dev_tensor(residues, torch.uint8, self.device)
        off = _dev_tensor(offsets, torch.int64, self.device)
        n = off.numel() - 1
        R = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
        bucket = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        order = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        boff = torch.empty(B + 1 if B > 0 else 1, dtype=torch.int32, device=self.device)
        self._check(lib().kd_decompose(self.handle, _ptr(res), _ptr(off), n, res.numel(), B, int(bool(globalized)),
                                       float(delta), _ptr(R), _ptr(bucket), _ptr(order), _ptr(boff)),
                    "kd_decompose")
        return dict(ranks=R[:n], bucket=bucket[:n], order=order[:n], offsets=boff)

    # ------------------------------------------- buckets and guide trees
    def gather_sequences(self, residues, offsets, order):
        """Sequences order[0..n) written back to back (redistribution):
        returns (residues, offsets) of the gathered set on the device."""
        res = _dev_tensor(residues, torch.uint8, self.device)
        off = _dev_tensor(offsets, torch.int64, self.device)
        idx = _dev_tensor(order, torch.int32, self.device)
        n = idx.numel()
        out = torch.empty(max(res.numel(), 1), dtype=torch.uint8, device=self.device)
        out_off = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        self._check(lib().kd_gather_sequences(self.handle, _ptr(res), _ptr(off), off.numel() - 1,
                                              res.numel(), _ptr(idx), n, _ptr(out), out.numel(),
                                              _ptr(out_off)), "kd_gather_sequences")
        return out[:res.numel()], out_off

    def distance_matrices(self, kset: KmerSet, delta: float = 0.1):
        """Equations 1-2 for every pair of every set: one flat f64 tensor,
        set s's n_s x n_s matrix after those of the sets before it."""
        first = kset.set_first()
        sizes = np.diff(first.astype(np.int64))
        D = torch.empty(max(int((sizes * sizes).sum()), 1), dtype=torch.float64, device=self.device)
        self._check(lib().kmer_distance_matrices(self.handle, kset.handle, float(delta), _ptr(D)),
                    "kmer_distance_matrices")
        return D[:int((sizes * sizes).sum())]

    def upgma(self, set_first, dist):
        """UPGMA guide tree of each set's matrix (layout of
        distance_matrices): (merges (sum n_s - 1, 2) int32, heights)."""
        sf = np.ascontiguousarray(np.asarray(set_first, dtype=np.uint32))
        D = _dev_tensor(dist, torch.float64, self.device)
        sizes = np.diff(sf.astype(np.int64))
        if sf.ndim != 1 or sf.size < 2 or D.numel() != int((sizes * sizes).sum()):
            raise ValueError("dist must hold the sets' n_s x n_s matrices back to back")
        m = int(sf[-1]) - (sf.size - 1)
        merges = torch.empty((max(m, 1), 2), dtype=torch.int32, device=self.device)
        heights = torch.empty(max(m, 1), dtype=torch.float64, device=self.device)
        self._check(lib().upgma_trees(self.handle, sf.size - 1, sf.ctypes.data_as(C.c_void_p), _ptr(D),
                                      _ptr(merges), _ptr(heights)), "upgma_trees")
        return merges[:m], heights[:m]

    def bucket_trees(self, residues, offsets, ranks, B: int, delta: float = 0.1):
        """The step after the split: the B buckets' sequences gathered, each
        bucket's distance matrix and UPGMA guide tree.  Returns dict(order,
        set_first (bucket bounds), dist, merges, heights)."""
        part = self.sample_partition(ranks, B)
        res, off = self.gather_sequences(residues, offsets, part["order"])
        first = u32(part["offsets"])
        kb = self.kmer_count_batch(res, off, first)
        try:
            D = self.distance_matrices(kb, delta)
        finally:
            kb.destroy()
        merges, heights = self.upgma(first, D)
        return dict(order=part["order"], set_first=first, dist=D, merges=merges, heights=heights)

    # ------------------------------------------------ profiles and PSP
    def psp_profile(self, aln):
        """Column frequencies of the 20 amino acids (ACDEFGHIKLMNPQRSTVWY) of
        an m x L alignment (uint8; '-' and '.' are gaps): (L, 20) f64."""
        A = _dev_tensor(aln, torch.uint8, self.device)
        if A.dim() != 2:
            raise ValueError("aln must be an m x L array")
        m, L = A.shape
        A = A.contiguous()
        f = torch.empty((max(L, 1), 20), dtype=torch.float64, device=self.device)
        self._check(lib().psp_profile(self.handle, _ptr(A), m, L, _ptr(f)), "psp_profile")
        return f[:L]

    def psp_scores(self, M, pairs, outs=None):
        """Equation 4 for every column pair of each (fx, fy) profile pair:
        a list of (lx, ly) f64 score tensors (written into `outs` when
        given)."""
        Md = _dev_tensor(M, torch.float64, self.device).contiguous()
        if Md.numel() != 400:
            raise ValueError("M must be 20 x 20")
        keep, res = [], []
        arr = (PspPair * max(len(pairs), 1))()
        for q, (fx, fy) in enumerate(pairs):
            X = _dev_tensor(fx, torch.float64, self.device).contiguous()
            Y = _dev_tensor(fy, torch.float64, self.device).contiguous()
            if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != 20 or Y.shape[1] != 20:
                raise ValueError("profiles must be L x 20")
            if outs is not None:
                S = outs[q]
                if (S.dtype != torch.float64 or tuple(S.shape) != (X.shape[0], Y.shape[0])
                        or not S.is_contiguous() or S.device != self.device):
                    raise ValueError("outs[%d] must be a contiguous (lx, ly) float64 device tensor" % q)
            else:
                S = torch.empty((X.shape[0], Y.shape[0]), dtype=torch.float64, device=self.device)
            keep += [X, Y]
            res.append(S)
            arr[q] = PspPair(X.data_ptr(), X.shape[0], Y.shape[0], Y.data_ptr(), S.data_ptr())
        self._check(lib().psp_scores(self.handle, _ptr(Md), len(pairs), C.cast(arr, C.c_void_p)),
                    "psp_scores")
        return res

    def psp_scores_packed(self, M, FX, lx, FY, ly, S=None):
        """psp_scores for profiles packed back to back: pair q is rows
        sum(lx[:q]) .. of FX (sum lx x 20) against rows sum(ly[:q]) .. of FY;
        its lx[q] x ly[q] scores go to S (flat, pair after pair).  Returns
        (S, offsets of each pair's scores)."""
        Md = _dev_tensor(M, torch.float64, self.device).contiguous()
        X = _dev_tensor(FX, torch.float64, self.device).contiguous()
        Y = _dev_tensor(FY, torch.float64, self.device).contiguous()
        lx = np.asarray(lx, dtype=np.int64)
        ly = np.asarray(ly, dtype=np.int64)
        if (Md.numel() != 400 or lx.shape != ly.shape or X.shape != (int(lx.sum()), 20)
                or Y.shape != (int(ly.sum()), 20) or (lx < 0).any() or (ly < 0).any()):
            raise ValueError("FX, FY must hold sum(lx), sum(ly) rows of 20; M must be 20 x 20")
        so = np.concatenate([[0], np.cumsum(lx * ly)])
        if S is None:
            S = torch.empty(max(int(so[-1]), 1), dtype=torch.float64, device=self.device)
        elif S.dtype != torch.float64 or S.numel() < int(so[-1]) or not S.is_contiguous():
            raise ValueError("S must be a contiguous float64 tensor of sum(lx * ly) entries")
        xo = np.concatenate([[0], np.cumsum(lx)[:-1]])
        yo = np.concatenate([[0], np.cumsum(ly)[:-1]])
        n = lx.size
        arr = np.zeros(max(n, 1), dtype=np.dtype([("fx", np.uint64), ("lx", np.uint32), ("ly", np.uint32),
                                                 ("fy", np.uint64), ("scores", np.uint64)]))
        arr["fx"][:n] = X.data_ptr() + 160 * xo
        arr["fy"][:n] = Y.data_ptr() + 160 * yo
        arr["lx"][:n] = lx
        arr["ly"][:n] = ly
        arr["scores"][:n] = S.data_ptr() + 8 * so[:-1]
        self._check(lib().psp_scores(self.handle, _ptr(Md), n, arr.ctypes.data_as(C.c_void_p)),
                    "psp_scores")
        return S, so

    # ------------------------------------------------------------ batches
    @staticmethod
    def _set_first(set_first, off):
        # the library cannot see device array sizes: the bounds must match here
        sf = np.ascontiguousarray(np.asarray(set_first, dtype=np.uint32))
        if sf.ndim != 1 or sf.size < 2 or int(sf[-1]) != off.numel() - 1:
            raise ValueError("set_first must have nsets+1 entries ending at the number of sequences")
        return sf

    @staticmethod
    def _host_u32(x, n, what):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.uint32))
        if a.ndim != 1 or a.size != n:
            raise ValueError(f"{what}: expected {n} entries, got {a.size}")
        return a

    def kmer_count_batch(self, residues, offsets, set_first) -> KmerSet:
        """Count many sets at once; set s = sequences set_first[s] .. set_first[s+1]-1."""
        res = _dev_tensor(residues, torch.uint8, self.device)
        off = _dev_tensor(offsets, torch.int64, self.device)
        sf = self._set_first(set_first, off)
        out = C.c_void_p()
        self._check(lib().kmer_count_batch(self.handle, _ptr(res), _ptr(off), res.numel(), sf.size - 1,
                                           sf.ctypes.data_as(C.c_void_p), C.byref(out)),
                    "kmer_count_batch")
        return KmerSet(self, out)

    def kmer_count_blocks(self, residues, offsets, B: int) -> KmerSet:
        """Algorithm 2 step 1: the B contiguous blocks of the input, each
        counted as its own set (the library computes the block bounds)."""
        res = _dev_tensor(residues, torch.uint8, self.device)
        off = _dev_tensor(offsets, torch.int64, self.device)
        out = C.c_void_p()
        self._check(lib().kmer_count_blocks(self.handle, _ptr(res), _ptr(off), off.numel() - 1, res.numel(),
                                            int(B), C.byref(out)), "kmer_count_blocks")
        return KmerSet(self, out)

    def sample_partition_batch(self, ranks, set_first, set_B, pivots: bool = True):
        R = _dev_tensor(ranks, torch.float64, self.device)
        sf = np.ascontiguousarray(np.asarray(set_first, dtype=np.uint32))
        if sf.ndim != 1 or sf.size < 2 or int(sf[-1]) != R.numel():
            raise ValueError("set_first must have nsets+1 entries ending at the number of ranks")
        nsets = sf.size - 1
        Bs = self._host_u32(set_B, nsets, "set_B")
        n = R.numel()
        nb, npv = int(Bs.astype(np.int64).sum()) + nsets, int(Bs.astype(np.int64).sum()) - nsets
        bucket = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        order = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        offsets = torch.empty(max(nb, 1), dtype=torch.int32, device=self.device)
        pr = torch.empty(max(npv, 1), dtype=torch.float64, device=self.device) if pivots else None
        pi = torch.empty(max(npv, 1), dtype=torch.int32, device=self.device) if pivots else None
        self._check(lib().sample_partition_batch(self.handle, _ptr(R), nsets, sf.ctypes.data_as(C.c_void_p),
                                                 Bs.ctypes.data_as(C.c_void_p), _ptr(bucket), _ptr(order),
                                                 _ptr(offsets), _ptr(pr), _ptr(pi)), "sample_partition_batch")
        out = dict(bucket=bucket[:n], order=order[:n], offsets=offsets[:nb])
        if pivots:
            out.update(pivot_rank=pr[:npv], pivot_idx=pi[:npv])
        return out

    def batch_run(self, residues, offsets, set_first, set_B, delta: float = 0.1, out=None):
        """Count, rank and split every set of a batch in one call.

        Returns dict(ranks f64[N], bucket, order (set-local), offsets
        (B_s + 1 per set, set after set)); `out` may supply those tensors."""
        res = _dev_tensor(residues, torch.uint8, self.device)
        off = _dev_tensor(offsets, torch.int64, self.device)
        sf = self._set_first(set_first, off)
        nsets = sf.size - 1
        Bs = self._host_u32(set_B, nsets, "set_B")
        n = off.numel() - 1
        nb = int(Bs.astype(np.int64).sum()) + nsets
        if out is None:
            out = dict(ranks=torch.empty(max(n, 1), dtype=torch.float64, device=self.device),
                       bucket=torch.empty(max(n, 1), dtype=torch.int32, device=self.device),
                       order=torch.empty(max(n, 1), dtype=torch.int32, device=self.device),
                       offsets=torch.empty(max(nb, 1), dtype=torch.int32, device=self.device))
        self._check(lib().kd_batch_run(self.handle, _ptr(res), _ptr(off), res.numel(), nsets,
                                       sf.ctypes.data_as(C.c_void_p), Bs.ctypes.data_as(C.c_void_p),
                                       float(delta), _ptr(out["ranks"]), _ptr(out["bucket"]),
                                       _ptr(out["order"]), _ptr(out["offsets"])), "kd_batch_run")
        return out

    def batch_plan(self, residues, offsets, set_first, set_B, delta: float = 0.1, out=None) -> "BatchPlan":
        """kd_batch_plan_create: the batch run once (outputs written) and
        captured as a graph; BatchPlan.launch() replays it."""
        res = _dev_tensor(residues, torch.uint8, self.device)
        off = _dev_tensor(offsets, torch.int64, self.device)
        sf = self._set_first(set_first, off)
        nsets = sf.size - 1
        Bs = self._host_u32(set_B, nsets, "set_B")
        n = off.numel() - 1
        nb = int(Bs.astype(np.int64).sum()) + nsets
        if out is None:
            out = dict(ranks=torch.empty(max(n, 1), dtype=torch.float64, device=self.device),
                       bucket=torch.empty(max(n, 1), dtype=torch.int32, device=self.device),
                       order=torch.empty(max(n, 1), dtype=torch.int32, device=self.device),
                       offsets=torch.empty(max(nb, 1), dtype=torch.int32, device=self.device))
        h = C.c_void_p()
        self._check(lib().kd_batch_plan_create(self.handle, _ptr(res), _ptr(off), res.numel(), nsets,
                                               sf.ctypes.data_as(C.c_void_p), Bs.ctypes.data_as(C.c_void_p),
                                               float(delta), _ptr(out["ranks"]), _ptr(out["bucket"]),
                                               _ptr(out["order"]), _ptr(out["offsets"]), C.byref(h)),
                    "kd_batch_plan_create")
        return BatchPlan(self, h, out)


class BatchPlan:
    """A batch captured as one HIP graph (kd_batch_plan_*): launch() replays
    count, rank and split of every set into the output tensors it holds."""

    def __init__(self, ctx: "Context", handle: C.c_void_p, out: dict):
        self.ctx, self.handle, self.out = ctx, handle, out

    @property
    def launches(self) -> int:
        return int(lib().kd_batch_plan_launches(self.handle))

    def launch(self):
        self.ctx._check(lib().kd_batch_plan_launch(self.handle), "kd_batch_plan_launch")
        return self.out

    def destroy(self):
        if getattr(self, "handle", None):
            lib().kd_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """Request server (kd_server_*): jobs are host arrays; results land in
    numpy arrays owned by this object until the job's record is polled."""

    def __init__(self, device: int = 0, hbm_budget: int = 200 << 30, max_batch_jobs: int = 0,
                 max_batch_seqs: int = 0, host_arena_bytes: int = 0, device_mirror: bool = True,
                 timeline: bool = False):
        L = lib()
        opts = ServerOpts(hbm_budget, max_batch_jobs, max_batch_seqs, host_arena_bytes,
                          0 if device_mirror else 1, 1 if timeline else 0)
        out = C.c_void_p()
        st = L.kd_server_create(device, C.byref(opts), C.byref(out))
        if st != KD_OK:
            raise KdError(st, "kd_server_create")
        self.handle = out
        self._live = {}  # ticket -> (inputs kept for the call, outputs)

    def submit(self, residues, offsets, B: int, delta: float = 0.1) -> int:
        res = np.ascontiguousarray(residues, dtype=np.uint8)
        off = np.ascontiguousarray(np.asarray(offsets).view(np.uint64) if np.asarray(offsets).dtype == np.int64
                                   else np.asarray(offsets, dtype=np.uint64))
        n = off.size - 1
        out = dict(ranks=np.empty(max(n, 1), np.float64), bucket=np.empty(max(n, 1), np.uint32),
                   order=np.empty(max(n, 1), np.uint32), offsets=np.empty(B + 1 if B > 0 else 1, np.uint32))
        job = Job(res.ctypes.data, off.ctypes.data, n, res.size, B, float(delta),
                  out["ranks"].ctypes.data, out["bucket"].ctypes.data, out["order"].ctypes.data,
                  out["offsets"].ctypes.data)
        t = C.c_uint64()
        st = lib().kd_server_submit(self.handle, C.byref(job), C.byref(t))
        if st != KD_OK:
            raise KdError(st, "kd_server_submit")
        for k in ("ranks", "bucket", "order"):
            out[k] = out[k][:n]
        self._live[int(t.value)] = out
        return int(t.value)

    def poll(self, max_records: int = 256, wait_s: float = 0.0):
        """List of dicts (ticket, status, batch_jobs, t_submit/start/done ns, and
        the result arrays when status is KD_OK)."""
        buf = (Done * max_records)()
        n = C.c_uint32()
        st = lib().kd_server_poll(self.handle, buf, max_records, C.byref(n), int(wait_s * 1e9))
        if st != KD_OK:
            raise KdError(st, "kd_server_poll")
        recs = []
        for d in buf[:n.value]:
            r = dict(ticket=int(d.ticket), status=int(d.status), batch_jobs=int(d.batch_jobs),
                     t_submit_ns=int(d.t_submit_ns), t_start_ns=int(d.t_start_ns), t_done_ns=int(d.t_done_ns))
            out = self._live.pop(r["ticket"], None)
            if out is not None and r["status"] == KD_OK:
                r.update(out)
            recs.append(r)
        return recs

    def cancel(self, ticket: int) -> int:
        """KD_OK, or the status code (KD_EBUSY: already running)."""
        return int(lib().kd_server_cancel(self.handle, ticket))

    def timeline(self, max_records: int = 65536):
        """Stage records of completed batches (kd_server_timeline), oldest first."""
        buf = (ServerStage * max_records)()
        n = C.c_uint32()
        st = lib().kd_server_timeline(self.handle, buf, max_records, C.byref(n))
        if st != KD_OK:
            raise KdError(st, "kd_server_timeline")
        return [dict(count=(b.count_start_ms, b.count_end_ms), rank=(b.rank_start_ms, b.rank_end_ms), jobs=b.jobs)
                for b in buf[:n.value]]

    def status(self):
        w, a, r, d = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32()
        res = C.c_uint64()
        lib().kd_server_status(self.handle, C.byref(w), C.byref(a), C.byref(r), C.byref(d), C.byref(res))
        return dict(waiting=w.value, admitted=a.value, running=r.value, done=d.value, reserved=res.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().kd_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = None


def default_context() -> Context:
    global _default
    if _default is None:
        _default = Context()
    return _default


def kmer_count(residues, offsets) -> KmerSet:
    return default_context().kmer_count(residues, offsets)


def kmer_similarity(kset, r0, nr, c0, nc, denom=False):
    return default_context().kmer_similarity(kset, r0, nr, c0, nc, denom)


def kmer_rank(kset, delta=0.1, out=None):
    return default_context().kmer_rank(kset, delta, out)


def sample_partition(ranks, B):
    return default_context().sample_partition(ranks, B)


def u16(t) -> np.ndarray:
    """CUDA int16-stored u16 tensor -> numpy uint16."""
    return t.cpu().numpy().view(np.uint16)


def u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)
