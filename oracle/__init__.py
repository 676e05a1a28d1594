"""CPU oracle (TEST INFRASTRUCTURE ONLY).

A plain, single-threaded C implementation of what the k-mer rank +
regular-sampling decomposition computes (``kd_oracle.c``), and this ctypes
wrapper.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import it; the GPU library never does, and the two share
no code.  Citations point at the paper's sections / equations; each C function
names the passage it follows.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
(worked examples, closed forms, brute force over the dense count vectors,
invariants).  The paper's Table 1 statistics cannot be reproduced (its data
set and Delta are not given), so they pin nothing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kd_oracle.c")
_lib = None

EPS = 46656
K_LEN = 6

ERRORS = {0: "ok", -1: "invalid argument", -2: "bad residue", -3: "sequence shorter than k",
          -4: "sequence has more than 65535 k-mers", -5: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code, seq=None, pos=None):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')}) seq={seq} pos={pos}")
        self.code, self.seq, self.pos = code, seq, pos


def _host_tag() -> str:
    """Short tag of the host CPU: the library is built with -march=native,
    so a copy built on one machine is never loaded on another."""
    import hashlib
    import platform
    sig = platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith(("model name", "flags")):
                    sig += line
                if line.startswith("flags"):
                    break
    except OSError:
        pass
    return hashlib.sha1(sig.encode()).hexdigest()[:12]


_LIB = os.path.join(_HERE, "liboracle-%s.so" % _host_tag())

# -O2 -march=native for the host it runs on; -ffp-contract=off keeps every
# multiply and add separately rounded (no FMA contraction), so the oracle's
# arithmetic is the same on every host.
CFLAGS = ["-O2", "-march=native", "-ffp-contract=off", "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (single-threaded C, flags in CFLAGS)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + ["-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_code.argtypes = [C.c_uint8]
        L.orc_code.restype = C.c_int
        L.orc_kmer_words.argtypes = [P, C.c_uint64, P, P]
        L.orc_kmer_words.restype = C.c_int64
        L.orc_count_dense.argtypes = [P, C.c_uint64, P]
        L.orc_count_dense.restype = C.c_int64
        L.orc_count_set.argtypes = [P, P, C.c_uint32, P, P, P, P, P, P]
        L.orc_count_set.restype = C.c_int
        L.orc_shared.argtypes = [P, P, C.c_uint64, P, P, C.c_uint64]
        L.orc_shared.restype = C.c_uint32
        L.orc_shared_dense.argtypes = [P, P]
        L.orc_shared_dense.restype = C.c_uint32
        L.orc_fraction.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_fraction.restype = C.c_double
        L.orc_distance.argtypes = [C.c_double, C.c_double]
        L.orc_distance.restype = C.c_double
        L.orc_similarity_block.argtypes = [P, P, P, P, C.c_uint32, C.c_uint32, C.c_uint32,
                                           C.c_uint32, P, P]
        L.orc_similarity_block.restype = None
        L.orc_rank_rows.argtypes = [P, P, P, P, C.c_uint32, P, C.c_uint32, C.c_double, P, P]
        L.orc_rank_rows.restype = None
        L.orc_partition.argtypes = [P, C.c_uint32, C.c_uint32, P, P, P, P, P]
        L.orc_partition.restype = C.c_int
        L.orc_local_ranks.argtypes = [P, P, P, P, C.c_uint32, C.c_uint32, C.c_double, P]
        L.orc_local_ranks.restype = C.c_int
        L.orc_global_samples.argtypes = [P, C.c_uint32, C.c_uint32, C.c_uint32, P]
        L.orc_global_samples.restype = C.c_int
        L.orc_global_rank_rows.argtypes = [P, P, P, P, P, C.c_uint32, P, C.c_uint32, C.c_double,
                                           P, P]
        L.orc_global_rank_rows.restype = None
        L.orc_distance_block.argtypes = [P, P, P, P, P, C.c_uint32, P, C.c_uint32, C.c_double, P]
        L.orc_distance_block.restype = None
        L.orc_upgma.argtypes = [P, C.c_uint32, P, P]
        L.orc_upgma.restype = C.c_int
        L.orc_profile.argtypes = [P, C.c_uint32, C.c_uint32, P, P]
        L.orc_profile.restype = C.c_int
        L.orc_psp.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P]
        L.orc_psp.restype = None
        L.orc_psp_matrix.argtypes = [P, P]
        L.orc_psp_matrix.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Lists:
    """Count vectors of a set as sorted nonzero entries (CSR)."""

    def __init__(self, ids, cnt, off, K):
        self.ids, self.cnt, self.off, self.K = ids, cnt, off, K

    @property
    def n(self):
        return int(self.K.shape[0])

    def entries(self, i):
        a, b = int(self.off[i]), int(self.off[i + 1])
        return self.ids[a:b], self.cnt[a:b]


def code(ch: int) -> int:
    return lib().orc_code(ch)


def kmer_words(seq: bytes) -> np.ndarray:
    s = np.frombuffer(seq, dtype=np.uint8).copy()
    out = np.zeros(max(len(seq), 1), dtype=np.uint32)
    bad = np.zeros(1, dtype=np.uint64)
    r = lib().orc_kmer_words(_p(s), len(seq), _p(out), _p(bad))
    if r < 0:
        raise OracleError(int(r), 0, int(bad[0]))
    return out[:r]


def count_dense(seq: bytes) -> np.ndarray:
    s = np.frombuffer(seq, dtype=np.uint8).copy()
    out = np.zeros(EPS, dtype=np.uint32)
    r = lib().orc_count_dense(_p(s), len(seq), _p(out))
    if r < 0:
        raise OracleError(int(r))
    return out


def count(ss) -> Lists:
    """Count vectors for a synth.SeqSet (or anything with residues/offsets)."""
    res = np.ascontiguousarray(ss.residues, dtype=np.uint8)
    off_in = np.ascontiguousarray(ss.offsets, dtype=np.uint64)
    N = off_in.shape[0] - 1
    cap = max(int(np.maximum(np.diff(off_in.astype(np.int64)) - (K_LEN - 1), 0).sum()), 1)
    ids = np.zeros(cap, dtype=np.uint16)
    cnt = np.zeros(cap, dtype=np.uint16)
    off = np.zeros(N + 1, dtype=np.uint64)
    K = np.zeros(max(N, 1), dtype=np.uint32)
    es = np.zeros(1, dtype=np.uint64)
    ep = np.zeros(1, dtype=np.uint64)
    r = lib().orc_count_set(_p(res), _p(off_in), N, _p(ids), _p(cnt), _p(off), _p(K), _p(es), _p(ep))
    if r != 0:
        raise OracleError(r, int(es[0]), int(ep[0]))
    tot = int(off[N])
    return Lists(ids[:tot].copy(), cnt[:tot].copy(), off, K[:N].copy())


def shared(L: Lists, i: int, j: int) -> int:
    ia, ca = L.entries(i)
    ib, cb = L.entries(j)
    ia, ca, ib, cb = (np.ascontiguousarray(x) for x in (ia, ca, ib, cb))
    return int(lib().orc_shared(_p(ia), _p(ca), len(ia), _p(ib), _p(cb), len(ib)))


def shared_dense(cx: np.ndarray, cy: np.ndarray) -> int:
    cx = np.ascontiguousarray(cx, dtype=np.uint32)
    cy = np.ascontiguousarray(cy, dtype=np.uint32)
    return int(lib().orc_shared_dense(_p(cx), _p(cy)))


def fraction(s: int, d: int) -> float:
    return float(lib().orc_fraction(s, d))


def distance(F: float, delta: float) -> float:
    return float(lib().orc_distance(F, delta))


def similarity(L: Lists, r0: int, nr: int, c0: int, nc: int):
    S = np.zeros((nr, nc), dtype=np.uint16)
    D = np.zeros((nr, nc), dtype=np.uint16)
    lib().orc_similarity_block(_p(L.ids), _p(L.cnt), _p(L.off), _p(L.K), r0, nr, c0, nc, _p(S), _p(D))
    return S, D


def rank(L: Lists, delta: float, rows=None, with_scale: bool = False):
    """Equation 3 for the given rows (all rows by default).  With
    ``with_scale`` also returns (1/N) sum_j |d(i,j)| per row."""
    N = L.n
    rows = np.arange(N, dtype=np.uint32) if rows is None else np.ascontiguousarray(rows, dtype=np.uint32)
    out = np.zeros(max(len(rows), 1), dtype=np.float64)
    sc = np.zeros(max(len(rows), 1), dtype=np.float64)
    lib().orc_rank_rows(_p(L.ids), _p(L.cnt), _p(L.off), _p(L.K), N, _p(rows), len(rows), delta,
                        _p(out), _p(sc))
    if with_scale:
        return out[:len(rows)], sc[:len(rows)]
    return out[:len(rows)]


def partition(R: np.ndarray, B: int):
    """Returns dict(bucket, order, offsets, pivot_rank, pivot_idx)."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    N = R.shape[0]
    bucket = np.zeros(max(N, 1), dtype=np.uint32)
    order = np.zeros(max(N, 1), dtype=np.uint32)
    offsets = np.zeros(B + 1 if B > 0 else 1, dtype=np.uint32)
    pr = np.zeros(max(B - 1, 1), dtype=np.float64)
    pi = np.zeros(max(B - 1, 1), dtype=np.uint32)
    r = lib().orc_partition(_p(R), N, B, _p(bucket), _p(order), _p(offsets), _p(pr), _p(pi))
    if r != 0:
        raise OracleError(r)
    return dict(bucket=bucket[:N], order=order[:N], offsets=offsets[:B + 1],
                pivot_rank=pr[:max(B - 1, 0)], pivot_idx=pi[:max(B - 1, 0)])


def local_ranks(L: Lists, B: int, delta: float):
    """Algorithm 2 steps 1-2: each of the B contiguous blocks ranked against
    itself (Equation 3 restricted to the block)."""
    out = np.zeros(max(L.n, 1), dtype=np.float64)
    r = lib().orc_local_ranks(_p(L.ids), _p(L.cnt), _p(L.off), _p(L.K), L.n, B, delta, _p(out))
    if r != 0:
        raise OracleError(r)
    return out[:L.n]


def global_samples(local: np.ndarray, B: int, k: int):
    """Algorithm 2 steps 3-5: k regular samples of each block's local-rank
    order, gathered block by block (input indices)."""
    local = np.ascontiguousarray(local, dtype=np.float64)
    out = np.zeros(max(B * k, 1), dtype=np.uint32)
    r = lib().orc_global_samples(_p(local), local.shape[0], B, k, _p(out))
    if r != 0:
        raise OracleError(r)
    return out[:B * k]


def global_rank(L: Lists, samples: np.ndarray, delta: float, rows=None, with_scale: bool = False):
    """Algorithm 2 step 6: the globalized rank of the given rows (all by
    default) against the gathered samples."""
    samples = np.ascontiguousarray(samples, dtype=np.uint32)
    rows = np.arange(L.n, dtype=np.uint32) if rows is None else np.ascontiguousarray(rows, dtype=np.uint32)
    if samples.size == 0 or (samples.size and int(samples.max()) >= L.n):
        raise OracleError(-1)
    out = np.zeros(max(len(rows), 1), dtype=np.float64)
    sc = np.zeros(max(len(rows), 1), dtype=np.float64)
    lib().orc_global_rank_rows(_p(L.ids), _p(L.cnt), _p(L.off), _p(L.K), _p(samples), samples.size,
                               _p(rows), len(rows), delta, _p(out), _p(sc))
    if with_scale:
        return out[:len(rows)], sc[:len(rows)]
    return out[:len(rows)]


def distance_block(L: Lists, rows, cols, delta: float):
    """Equations 1-2 for the pairs rows x cols (sequence indices)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    cols = np.ascontiguousarray(cols, dtype=np.uint32)
    out = np.zeros((max(rows.size, 1), max(cols.size, 1)), dtype=np.float64)
    lib().orc_distance_block(_p(L.ids), _p(L.cnt), _p(L.off), _p(L.K), _p(rows), rows.size, _p(cols),
                             cols.size, delta, _p(out))
    return out[:rows.size, :cols.size]


def distance_matrix(L: Lists, idx, delta: float):
    """Equations 1-2 for every ordered pair of the sequences idx (n x n)."""
    return distance_block(L, idx, idx, delta)


def upgma(d: np.ndarray):
    """UPGMA guide tree of a dissimilarity matrix: (merges (n-1, 2) int32,
    heights (n-1,) float64); see orc_upgma for the slot and tie rules."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.shape[0]
    if d.ndim != 2 or d.shape[1] != n:
        raise OracleError(-1)
    merges = np.zeros((max(n - 1, 1), 2), dtype=np.int32)
    heights = np.zeros(max(n - 1, 1), dtype=np.float64)
    r = lib().orc_upgma(_p(d), n, _p(merges), _p(heights))
    if r != 0:
        raise OracleError(r)
    return merges[:n - 1], heights[:n - 1]


AMINO = b"ACDEFGHIKLMNPQRSTVWY"


def profile(aln: np.ndarray):
    """Column frequencies of the 20 amino acids (order AMINO) of an m x L
    alignment (uint8 rows; '-' and '.' are gaps): (L, 20) float64."""
    aln = np.ascontiguousarray(aln, dtype=np.uint8)
    m, L = aln.shape
    f = np.zeros((max(L, 1), 20), dtype=np.float64)
    bad = C.c_uint64(0)
    r = lib().orc_profile(_p(aln), m, L, _p(f), C.byref(bad))
    if r != 0:
        raise OracleError(r, pos=int(bad.value))
    return f[:L]


def psp(fx: np.ndarray, fy: np.ndarray, M: np.ndarray):
    """Equation 4 for every column pair of two profiles: (Lx, Ly)."""
    fx = np.ascontiguousarray(fx, dtype=np.float64)
    fy = np.ascontiguousarray(fy, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    S = np.zeros((max(fx.shape[0], 1), max(fy.shape[0], 1)), dtype=np.float64)
    lib().orc_psp(_p(fx), fx.shape[0], _p(fy), fy.shape[0], _p(M), _p(S))
    return S[:fx.shape[0], :fy.shape[0]]


def psp_matrix(P: np.ndarray):
    """log(P_ij / (p_i p_j)) with p_i = sum_j P_ij (Equation 4's log term)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    M = np.zeros((20, 20), dtype=np.float64)
    r = lib().orc_psp_matrix(_p(P), _p(M))
    if r != 0:
        raise OracleError(r)
    return M

