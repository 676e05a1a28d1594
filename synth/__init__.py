"""Seeded synthetic protein-family generator.

This module only draws inputs.  It holds none of the method's arithmetic
(no k-mer encoding, no similarity, no ranking, no sampling); the CPU oracle
and the GPU library both consume what it returns.

The paper evaluates on sets made with the Rose sequence generator
(Section 4.1, "Rose" experiments) plus BaliBase, Prefab and a Pfam family;
none of those are available here, so this star-phylogeny generator stands in
for them.  Every family is a random ancestor drawn uniformly over the 20
standard amino acids; members are derived by per-site substitution
(probability ``r``, replaced by a uniformly chosen *different* residue) and
per-site indel events (probability ``indel``; insertion or deletion with
probability 1/2 each; event length geometric with p = 1/3, mean 3; inserted
residues uniform).  Family sizes are floor(N/F), the first N mod F families
getting one extra member, and the whole set is shuffled.

Workloads (sizes as used throughout the tests and the benchmark):

* ``small``      N=512, 8 families, ancestor length U[200,400], r=0.10.
* ``paper20k``   N=20,000, 200 families, lognormal lengths (mean 350,
                 sigma 0.5 in log space, clipped to [50,2000]),
                 r ~ U[0.05,0.30] per family.
* ``large100k``  N=100,000, 1,000 families, lognormal mean 300,
                 r ~ U[0.05,0.40].
* ``batched``    4,096 independent sets, N = round(exp U[ln 32, ln 2048]),
                 families U{4..32} (capped at N), lognormal mean 300,
                 r ~ U[0.05,0.30], B = min(8, N // 32).
* ``served``     request stream; N log-uniform in [64, 8192], lognormal
                 mean 300, families U{4..32}, B = max(1, N // 256),
                 Poisson arrivals.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

AMINO = np.frombuffer(b"ACDEFGHIKLMNPQRSTVWY", dtype=np.uint8).copy()
LOGN_SIGMA = 0.5
INDEL_RATE = 0.02
INDEL_GEOM_P = 1.0 / 3.0


@dataclasses.dataclass
class SeqSet:
    """A set of sequences as one packed ASCII buffer plus CSR offsets."""

    residues: np.ndarray  # uint8 [sum n], ASCII upper-case amino acids
    offsets: np.ndarray   # uint64 [N+1]
    family: np.ndarray    # int32 [N], generating family (bookkeeping only)
    name: str = ""
    B: int = 1            # bucket count the workload asks for

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def seq(self, i: int) -> bytes:
        return self.residues[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)


def from_strings(seqs, name: str = "", B: int = 1) -> SeqSet:
    """Pack a list of str/bytes into a SeqSet (used by tiny hand-made cases)."""
    bs = [s.encode() if isinstance(s, str) else bytes(s) for s in seqs]
    lens = np.array([len(b) for b in bs], dtype=np.uint64)
    off = np.zeros(len(bs) + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    res = np.frombuffer(b"".join(bs), dtype=np.uint8).copy() if bs else np.zeros(0, np.uint8)
    return SeqSet(res, off, np.zeros(len(bs), np.int32), name, B)


def _lognormal_lengths(rng, count, mean, lo=50, hi=2000):
    mu = math.log(mean) - LOGN_SIGMA ** 2 / 2.0
    x = rng.lognormal(mu, LOGN_SIGMA, size=count)
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def _derive_members(rng, anc: np.ndarray, m: int, r: float, indel: float):
    """Derive ``m`` members from ancestor codes ``anc`` (values 0..19).

    Returns (codes concatenated, lengths).  Vectorised over members: the
    per-(member, site) emission count is 'inserted residues before the
    site' + 'site kept', and the output is one np.repeat over all sites.
    """
    L = anc.shape[0]
    base = np.broadcast_to(anc, (m, L)).copy()
    sub = rng.random((m, L)) < r
    nsub = int(sub.sum())
    base[sub] = (base[sub] + rng.integers(1, 20, size=nsub)) % 20
    ev = rng.random((m, L)) < indel
    is_ins = rng.random((m, L)) < 0.5
    glen = rng.geometric(INDEL_GEOM_P, size=(m, L))
    pos = np.arange(L, dtype=np.int64)[None, :]
    del_until = np.where(ev & ~is_ins, pos + glen, -1)
    reach = np.maximum.accumulate(del_until, axis=1)
    kept = ~(reach > pos)
    ins_len = np.where(ev & is_ins, glen, 0)
    emit = (ins_len + kept).ravel()
    total = int(emit.sum())
    site = np.repeat(np.arange(m * L, dtype=np.int64), emit)
    start = np.cumsum(emit) - emit
    within = np.arange(total, dtype=np.int64) - np.repeat(start, emit)
    flat_ins = ins_len.ravel()
    is_orig = kept.ravel()[site] & (within == flat_ins[site])
    out = rng.integers(0, 20, size=total).astype(np.uint8)
    out[is_orig] = base.ravel()[site[is_orig]].astype(np.uint8)
    lens = (ins_len + kept).sum(axis=1).astype(np.int64)
    # Guard the k-mer length floor: a member shorter than 6 residues cannot
    # occur for ancestors of >= 50 sites in practice; pad deterministically.
    if lens.min(initial=6) < 6:
        pieces, o = [], 0
        for ln in lens:
            p = out[o:o + ln]
            o += ln
            if ln < 6:
                p = np.concatenate([p, rng.integers(0, 20, size=6 - ln).astype(np.uint8)])
            pieces.append(p)
        out = np.concatenate(pieces)
        lens = np.maximum(lens, 6)
    return out, lens


def families(rng, N: int, F: int, anc_lengths: np.ndarray, rates: np.ndarray,
             indel: float = INDEL_RATE, name: str = "", B: int = 1) -> SeqSet:
    F = max(1, min(F, N))
    sizes = np.full(F, N // F, dtype=np.int64)
    sizes[: N % F] += 1
    codes, lens, fam = [], [], []
    for f in range(F):
        anc = rng.integers(0, 20, size=int(anc_lengths[f])).astype(np.uint8)
        c, ln = _derive_members(rng, anc, int(sizes[f]), float(rates[f]), indel)
        codes.append(c)
        lens.append(ln)
        fam.append(np.full(int(sizes[f]), f, dtype=np.int32))
    codes = np.concatenate(codes)
    lens = np.concatenate(lens)
    fam = np.concatenate(fam)
    # shuffle whole sequences
    perm = rng.permutation(N)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    lens_p = lens[perm]
    new_starts = np.cumsum(lens_p) - lens_p
    total = int(lens_p.sum())
    idx = np.arange(total, dtype=np.int64) + np.repeat(starts[perm] - new_starts, lens_p)
    res = AMINO[codes[idx]]
    off = np.zeros(N + 1, dtype=np.uint64)
    np.cumsum(lens_p, out=off[1:])
    return SeqSet(res, off, fam[perm], name, B)


def small(seed: int = 1) -> SeqSet:
    rng = np.random.default_rng(seed)
    F = 8
    lens = rng.integers(200, 401, size=F)
    rates = np.full(F, 0.10)
    return families(rng, 512, F, lens, rates, name="small-512", B=4)


def paper20k(seed: int = 2, N: int = 20000) -> SeqSet:
    rng = np.random.default_rng(seed)
    F = max(1, N // 100)
    lens = _lognormal_lengths(rng, F, 350)
    rates = rng.uniform(0.05, 0.30, size=F)
    return families(rng, N, F, lens, rates, name=f"paper-{N}", B=16)


def large100k(seed: int = 3, N: int = 100000) -> SeqSet:
    rng = np.random.default_rng(seed)
    F = max(1, N // 100)
    lens = _lognormal_lengths(rng, F, 300)
    rates = rng.uniform(0.05, 0.40, size=F)
    return families(rng, N, F, lens, rates, name=f"large-{N}", B=64)


def batch_set(seq: np.random.SeedSequence) -> SeqSet:
    rng = np.random.default_rng(seq)
    N = int(round(math.exp(rng.uniform(math.log(32), math.log(2048)))))
    F = min(int(rng.integers(4, 33)), N)
    lens = _lognormal_lengths(rng, F, 300)
    rates = rng.uniform(0.05, 0.30, size=F)
    return families(rng, N, F, lens, rates, name=f"batch-{N}", B=min(8, N // 32))


def batched(seed: int = 4, nsets: int = 4096, workers: int = 1):
    """The batched workload: ``nsets`` independent sets (list of SeqSet).

    Set s is drawn from child s of ``SeedSequence(seed)``, so the result does
    not depend on ``workers`` (processes forked to draw sets in parallel;
    call this before the process initializes a GPU)."""
    children = np.random.SeedSequence(seed).spawn(nsets)
    if workers <= 1 or nsets < 2 * workers:
        return [batch_set(c) for c in children]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(batch_set, children, chunksize=max(1, nsets // (8 * workers)))


def concat(sets):
    """Lay several SeqSets end to end.

    Returns (residues u8, offsets u64[sum N + 1], set_first u32[len(sets)+1],
    B u32[len(sets)]): set s is sequences set_first[s] .. set_first[s+1]-1."""
    ns = np.array([x.offsets.size - 1 for x in sets], dtype=np.int64)
    first = np.zeros(len(sets) + 1, dtype=np.uint32)
    np.cumsum(ns, out=first[1:])
    res = np.concatenate([x.residues for x in sets]) if sets else np.zeros(0, np.uint8)
    tot = np.cumsum([0] + [int(x.residues.size) for x in sets[:-1]]).astype(np.uint64)
    off = np.zeros(int(first[-1]) + 1, dtype=np.uint64)
    for q, x in enumerate(sets):
        off[int(first[q]):int(first[q + 1])] = x.offsets[:-1] + tot[q]
    off[-1] = res.size
    Bs = np.array([x.B for x in sets], dtype=np.uint32)
    return res, off, first, Bs


def served_job(seq: np.random.SeedSequence, nmin: int = 64, nmax: int = 8192) -> SeqSet:
    rng = np.random.default_rng(seq)
    N = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    F = min(int(rng.integers(4, 33)), N)
    lens = _lognormal_lengths(rng, F, 300)
    rates = rng.uniform(0.05, 0.30, size=F)
    return families(rng, N, F, lens, rates, name=f"job-{N}", B=max(1, N // 256))


def _served_job_default(seq):
    return served_job(seq)


def served_jobs(seed: int = 5, njobs: int = 1000, workers: int = 1):
    """The jobs of the served workload (independent of the arrival rate)."""
    job_seqs = np.random.SeedSequence(seed).spawn(njobs + 1)[1:]
    if workers <= 1 or njobs < 2 * workers:
        return [served_job(s) for s in job_seqs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_served_job_default, job_seqs, chunksize=max(1, njobs // (8 * workers)))


def served_arrivals(seed: int = 5, njobs: int = 1000, rate: float = 100.0) -> np.ndarray:
    """Poisson arrival times (seconds) of the served workload at `rate` jobs/s."""
    arr_seq = np.random.SeedSequence(seed).spawn(njobs + 1)[0]
    rng = np.random.default_rng(arr_seq)
    return np.cumsum(rng.exponential(1.0 / rate, size=njobs))


def served_stream(seed: int = 5, njobs: int = 1000, rate: float = 100.0,
                  nmin: int = 64, nmax: int = 8192):
    """Poisson request stream: list of (arrival_seconds, SeqSet)."""
    ss = np.random.SeedSequence(seed)
    job_seqs = ss.spawn(njobs + 1)[1:]
    t = served_arrivals(seed, njobs, rate)
    return [(float(t[i]), served_job(job_seqs[i], nmin, nmax)) for i in range(njobs)]


def random_tiny(rng, N: int, lo: int = 6, hi: int = 60, alphabet: bytes = b"ACDEFGHIKLMNPQRSTVWY") -> SeqSet:
    """Unstructured random sequences for tiny brute-force checks."""
    al = np.frombuffer(alphabet, dtype=np.uint8)
    seqs = [al[rng.integers(0, len(al), size=int(rng.integers(lo, hi + 1)))].tobytes() for _ in range(N)]
    return from_strings(seqs, name=f"tiny-{N}")


CONFIGS = {
    "small": small,
    "paper20k": paper20k,
    "large100k": large100k,
}


def rank_like(N: int, seed: int, spread: float = 0.06, center: float = 2.0,
              tie_frac: float = 0.05) -> np.ndarray:
    """Synthetic k-mer-rank-shaped values for exercising the decomposition at
    full size without computing ranks: a few tight clusters (one per family
    group) around ``center``, with ``tie_frac`` of the entries made exact
    duplicates of other entries so that index tie-breaking matters."""
    rng = np.random.default_rng(seed)
    nclus = max(1, N // 100)
    mu = center + spread * rng.standard_normal(nclus)
    R = mu[rng.integers(0, nclus, size=N)] + 0.2 * spread * rng.standard_normal(N)
    k = int(tie_frac * N)
    if k and N > 1:
        dst = rng.integers(0, N, size=k)
        src = rng.integers(0, N, size=k)
        R[dst] = R[src]
    return R.astype(np.float64)
