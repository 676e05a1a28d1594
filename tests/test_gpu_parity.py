"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars: word lists and shared counts bit-exact; ranks within
1e-12 * (1/N) sum_j |d(i,j)| (the oracle returns that scale); buckets
identical (bit-exact when both sides see the same ranks, and otherwise
identical except for keys within twice the rank tolerance of a pivot).
"""
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_1744_amd as kd
    kd.lib()  # raises if the library is missing: no fallback
    return kd


@pytest.fixture(scope="module")
def ctx(kd):
    c = kd.Context()
    yield c
    c.synchronize()


def gpu_lists(kd, ctx, ss):
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    ids, cnt, off = kset.export_lists()
    return kset, kd.u16(ids), kd.u16(cnt), off.cpu().numpy().astype(np.uint64)


def check_lists(kd, ctx, ss, L):
    kset, ids, cnt, off = gpu_lists(kd, ctx, ss)
    assert kset.n == ss.n
    assert np.array_equal(off, L.off)
    assert np.array_equal(ids, L.ids)
    assert np.array_equal(cnt, L.cnt)
    return kset


def check_ranks(R_gpu, R_or, scale):
    err = np.abs(R_gpu - R_or)
    bad = err > RTOL * scale
    assert not bad.any(), (np.flatnonzero(bad)[:10], err[bad][:10], scale[bad][:10])


# ------------------------------------------------------------- counting --

@pytest.mark.parametrize("name", ["small", "tiny-AC", "tiny-AA", "ragged-77"])
def test_count_lists(kd, ctx, oracle_mod, name):
    rng = np.random.default_rng(21)
    if name == "small":
        ss = synth.small()
    elif name == "tiny-AC":
        ss = synth.random_tiny(rng, 40, 6, 300, b"AC")
    elif name == "tiny-AA":
        ss = synth.random_tiny(rng, 40, 6, 120, b"AGC")
    else:
        ss = synth.random_tiny(rng, 77, 6, 700)
    say("count", name, ss.n)
    check_lists(kd, ctx, ss, oracle_mod.count(ss))


def test_count_long_sequences(kd, ctx, oracle_mod):
    """Sequences above the one-wave limit (4096 words) take the dense-LDS
    path; 65540 residues is the longest allowed (65535 words)."""
    rng = np.random.default_rng(22)
    al = np.frombuffer(b"ACDEFGHIKLMNPQRSTVWY", dtype=np.uint8)
    seqs = [al[rng.integers(0, 20, size=n)].tobytes() for n in (4101, 4102, 9000, 300)]
    seqs += [b"A" * 65540, b"ACDEFGHIKL" * 700, b"CCCCCC"]
    ss = synth.from_strings(seqs)
    say("count-long", [len(s) for s in seqs])
    check_lists(kd, ctx, ss, oracle_mod.count(ss))


@pytest.mark.parametrize("alphabet", [b"ACDEFGHIKLMNPQRSTVWY", b"AC"])
def test_count_path_boundaries(kd, ctx, oracle_mod, alphabet):
    """Sequence sizes at every boundary of the counting paths: one wave with
    1, 2 or 4 residues per lane and the register sort (n <= 64, 128, 256
    residues), one wave with 8 or 16 per lane and the LDS bitmap (n <= 512,
    1024), the 4096-word pass and the dense-histogram pass (K = n - 5 words);
    the two-letter alphabet makes almost every word repeat."""
    rng = np.random.default_rng(24)
    al = np.frombuffer(alphabet, dtype=np.uint8)
    Ks = [1, 2, 59, 60, 63, 64, 65, 123, 124, 127, 128, 129, 251, 252, 255, 256, 257, 507, 508,
          511, 512, 513, 1019, 1020, 1023, 1024, 1025, 2048, 4095, 4096, 4097]
    seqs = [al[rng.integers(0, len(al), size=k + 5)].tobytes() for k in Ks]
    ss = synth.from_strings(seqs)
    say("count-boundaries", alphabet[:4], len(seqs))
    check_lists(kd, ctx, ss, oracle_mod.count(ss))


@pytest.mark.parametrize("N", [200_000, 800_000])
def test_count_bitmap_pass_large_sets(kd, ctx, oracle_mod, N):
    """Sets large enough for the LDS-bitmap pass (N >= 64 x its resident
    waves, 196,608 on 256 compute units): at 200,000 one wave per chunk of
    16 sequences, at 800,000 (>= 256 x the waves) a persistent launch that
    takes chunks of 64 from its counter.  Most sequences have 257..1024
    residues (that pass's range).  Word lists of 3,000 sampled sequences
    bit-exact against the oracle."""
    rng = np.random.default_rng(31)
    lens = np.where(rng.random(N) < 0.9, rng.integers(257, 601, N), rng.integers(6, 1101, N))
    off = np.zeros(N + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    al = np.frombuffer(b"ACDEFGHIKLMNPQRSTVWY", dtype=np.uint8)
    res = al[rng.integers(0, 20, size=int(off[-1]), dtype=np.uint8)]
    ss = synth.SeqSet(res, off, np.zeros(N, dtype=np.int32), f"bitmap-{N}")
    say("count-bitmap-pass", N, int(off[-1]))
    kset, ids, cnt, goff = gpu_lists(kd, ctx, ss)
    assert kset.n == N
    rows = np.sort(rng.choice(N, size=3000, replace=False))
    L = oracle_mod.count(synth.from_strings([ss.seq(int(i)) for i in rows]))
    for j, i in enumerate(rows):
        a, b = int(goff[i]), int(goff[i + 1])
        c, d = int(L.off[j]), int(L.off[j + 1])
        assert np.array_equal(ids[a:b], L.ids[c:d]) and np.array_equal(cnt[a:b], L.cnt[c:d]), int(i)
    # a residue that is not an amino acid in two sequences on the bitmap
    # path: the first sequence's first bad position is reported
    on = np.flatnonzero((lens > 256) & (lens <= 1024))
    i0, i1 = int(on[N // 3 % len(on)]), int(on[-1])
    res[int(off[i1]) + 7] = ord("Z")
    res[int(off[i0]) + 200] = ord("*")
    res[int(off[i0]) + 250] = ord("b")
    say("count-bitmap-pass error", i0, i1)
    with pytest.raises(kd.KdError) as e:
        ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    assert e.value.status == -2 and e.value.seq == i0 and e.value.pos == 200


def test_count_errors(kd, ctx):
    cases = [
        (["ACDEFGH", "ACDXFGH", "ACDEFGH"], -2, 1, 3),
        (["ACDEFGH", "ACDEFG", "ACDEF"], -3, 2, None),
        (["ACDEFGH", "ACDEFGH", "A" * 65541], -4, 2, None),
        (["ACDEFGH", "acdefgh"], -2, 1, 0),
        (["ACDEFGH", "B" * 5000], -2, 1, 0),   # bad residue on the long path
        (["ACDEFGH" * 40, "ACDEFGH" * 40 + "Z"], -2, 1, 280),  # last residue, bitmap path
        (["ACDEFGH" * 36 + "ACDZ"], -2, 0, 255),  # last residue, register path (256 residues)
        (["ACDEFGH" * 146 + "AX"], -2, 0, 1023),  # last residue, 16 residues per lane
        (["ACDEFGH" * 50 + "QQ*QQ*" + "ACDEFGH" * 20], -2, 0, 352),  # the first of two
        (["ACDEFGH", "x" + "ACDEFGH" * 60], -2, 1, 0),  # first residue, bitmap path
        (["ACDEFGH" * 300 + "*" + "ACDEFGH"], -2, 0, 2100),  # the 4096-word path
        (["ACDEFGHIK", "ACDEFGHIK" * 30, "ACDEFGHIK", "ACDEFG1"], -2, 3, 6),
    ]
    for seqs, code, seq, pos in cases:
        say("count-error", code, seq)
        ss = synth.from_strings(seqs)
        with pytest.raises(kd.KdError) as e:
            ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
        assert e.value.status == code and e.value.seq == seq
        if pos is not None:
            assert e.value.pos == pos
    # the context keeps working after errors
    ss = synth.from_strings(["ACDEFGHIK", "ACDEFG"])
    assert ctx.kmer_count(ss.residues, ss.offsets.view(np.int64)).n == 2


def test_count_empty_set(kd, ctx):
    import torch
    kset = ctx.kmer_count(torch.zeros(0, dtype=torch.uint8), torch.zeros(1, dtype=torch.int64))
    assert kset.n == 0 and kset.entries == 0
    R = ctx.kmer_rank(kset, 0.1)
    assert R.numel() == 0


def test_export_dense(kd, ctx, oracle_mod):
    ss = synth.random_tiny(np.random.default_rng(23), 9, 6, 200, b"ACDEF")
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    dense = kd.u16(kset.export_dense(2, 5))
    for q in range(5):
        ref = oracle_mod.count_dense(ss.seq(2 + q))
        assert np.array_equal(dense[q].astype(np.uint32), ref)


# ----------------------------------------------------------- similarity --

@pytest.mark.parametrize("name", ["small", "tiny-AC", "tiny-ACD", "ragged-77", "repeats"])
def test_similarity_full_block(kd, ctx, oracle_mod, name):
    rng = np.random.default_rng(31)
    if name == "small":
        ss = synth.small()
    elif name == "tiny-AC":
        ss = synth.random_tiny(rng, 50, 6, 400, b"AC")
    elif name == "tiny-ACD":
        ss = synth.random_tiny(rng, 70, 6, 200, b"ACD")
    elif name == "ragged-77":
        ss = synth.random_tiny(rng, 77, 6, 700)
    else:  # low-complexity sequences: counts far above 2 on both sides
        ss = synth.from_strings([b"A" * int(n) + b"C" * int(m) for n, m in rng.integers(6, 3000, size=(33, 2))]
                                + [b"AC" * 900, b"A" * 4000])
    L = oracle_mod.count(ss)
    S_or, D_or = oracle_mod.similarity(L, 0, ss.n, 0, ss.n)
    say("similarity", name, ss.n)
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    S, Dn = ctx.kmer_similarity(kset, 0, ss.n, 0, ss.n, denom=True)
    S, Dn = kd.u16(S), kd.u16(Dn)
    assert np.array_equal(Dn, D_or)
    bad = np.argwhere(S != S_or)
    assert bad.size == 0, (bad[:10], S[tuple(bad[:5].T)], S_or[tuple(bad[:5].T)])


def test_similarity_offset_blocks(kd, ctx, oracle_mod):
    ss = synth.small()
    L = oracle_mod.count(ss)
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    for r0, nr, c0, nc in [(3, 29, 100, 411), (511, 1, 0, 512), (0, 512, 7, 1), (200, 40, 200, 40)]:
        say("similarity-block", r0, nr, c0, nc)
        S = kd.u16(ctx.kmer_similarity(kset, r0, nr, c0, nc))
        assert np.array_equal(S, oracle_mod.similarity(L, r0, nr, c0, nc)[0])
    with pytest.raises(kd.KdError):
        ctx.kmer_similarity(kset, 500, 13, 0, 1)


# ----------------------------------------------------------------- rank --

@pytest.mark.parametrize("name,delta", [("small", 0.1), ("small", 1e-3), ("tiny-AC", 0.1),
                                        ("ragged-77", 0.1), ("ragged-1000", 0.5)])
def test_rank_full(kd, ctx, oracle_mod, name, delta):
    rng = np.random.default_rng(41)
    if name == "small":
        ss = synth.small()
    elif name == "tiny-AC":
        ss = synth.random_tiny(rng, 50, 6, 400, b"AC")
    elif name == "ragged-77":
        ss = synth.random_tiny(rng, 77, 6, 700)
    else:
        s = synth.paper20k(seed=9, N=1000)
        ss = synth.from_strings([s.seq(i) for i in range(997)])
    L = oracle_mod.count(ss)
    R_or, scale = oracle_mod.rank(L, delta, with_scale=True)
    say("rank", name, ss.n, delta)
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    R = ctx.kmer_rank(kset, delta).cpu().numpy()
    check_ranks(R, R_or, scale)


def test_rank_closed_forms(kd, ctx):
    """Closed forms of Equation 3.  Delta + F is rounded once before the log
    (up to 1.1e-16 absolute in d) and tile partial sums round once more, so
    the bar is 1e-13 relative: 10x tighter than the parity tolerance."""
    say("rank-closed-forms")
    delta, rel = 0.1, 1e-13
    ss = synth.from_strings(["AAAAAAA", "GPSTAG", "CCCCCC"])
    R = ctx.kmer_rank(ctx.kmer_count(ss.residues, ss.offsets.view(np.int64)), delta).cpu().numpy()
    # X and Y tie exactly in the reals; the tile partial sums group their
    # terms differently, so the GPU tie holds to rounding, not bitwise
    assert R[0] == pytest.approx(R[1], rel=rel)
    assert R[0] == pytest.approx((2 * -math.log1p(delta) - math.log(delta)) / 3, rel=rel)
    assert R[2] == pytest.approx((2 * -math.log(delta) - math.log1p(delta)) / 3, rel=rel)
    ss = synth.from_strings(["MKVLAAGIVGLLLAQ"] * 37)
    R = ctx.kmer_rank(ctx.kmer_count(ss.residues, ss.offsets.view(np.int64)), delta).cpu().numpy()
    np.testing.assert_allclose(R, -math.log1p(delta), rtol=rel, atol=0)
    ss = synth.from_strings(["ACDEFGHIKLMNPQ"])
    R = ctx.kmer_rank(ctx.kmer_count(ss.residues, ss.offsets.view(np.int64)), delta).cpu().numpy()
    assert R[0] == pytest.approx(-math.log1p(delta), rel=rel)
    # pairwise-disjoint word sets: ((N-1)(-ln D) - ln(1+D)) / N
    seqs = ["AAAAAAAA", "CCCCCC", "DDDDDDDDDDD", "FFFFFFF", "HHHHHH", "IIIIIIIIIIIIIII",
            "ACACACACAC", "DFDFDFDFDF"]
    ss = synth.from_strings(seqs)
    R = ctx.kmer_rank(ctx.kmer_count(ss.residues, ss.offsets.view(np.int64)), delta).cpu().numpy()
    N = len(seqs)
    np.testing.assert_allclose(R, ((N - 1) * -math.log(delta) - math.log1p(delta)) / N, rtol=rel, atol=0)


def test_rank_deterministic(kd, ctx):
    ss = synth.small()
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    a = ctx.kmer_rank(kset, 0.1).cpu().numpy()
    b = ctx.kmer_rank(kset, 0.1).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    # a fresh set of the same input gives the same bits
    c = ctx.kmer_rank(ctx.kmer_count(ss.residues, ss.offsets.view(np.int64)), 0.1).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), c.view(np.uint64))


def test_rank_errors(kd, ctx):
    ss = synth.small()
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    for d in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(kd.KdError):
            ctx.kmer_rank(kset, d)
    other = kd.Context()  # a set belongs to the context that counted it
    try:
        with pytest.raises(kd.KdError):
            other.kmer_rank(kset, 0.1)
        with pytest.raises(kd.KdError):
            other.kmer_similarity(kset, 0, 2, 0, 2)
    finally:
        other.close()


# ------------------------------------------------------------ partition --

def check_partition_equal(kd, p_gpu, p_or, B):
    assert np.array_equal(kd.u32(p_gpu["bucket"]), p_or["bucket"])
    assert np.array_equal(kd.u32(p_gpu["order"]), p_or["order"])
    assert np.array_equal(kd.u32(p_gpu["offsets"]), p_or["offsets"])
    assert np.array_equal(kd.u32(p_gpu["pivot_idx"]), p_or["pivot_idx"])
    assert np.array_equal(p_gpu["pivot_rank"].cpu().numpy(), p_or["pivot_rank"])


def test_partition_golden(kd, ctx):
    from conftest import golden_lines
    cur = None
    for line in golden_lines("partition_cases.txt"):
        k, *v = line.split()
        if k == "case":
            cur = {}
        elif k == "end":
            R = np.array([float(x) for x in cur["ranks"]])
            B = int(cur["B"][0])
            say("partition-golden", B, len(R))
            p = ctx.sample_partition(R, B)
            assert list(kd.u32(p["bucket"])) == [int(x) for x in cur["bucket"]]
            assert list(kd.u32(p["offsets"])) == [int(x) for x in cur["offsets"]]
            assert list(kd.u32(p["order"])) == [int(x) for x in cur["order"]]
            assert list(kd.u32(p["pivot_idx"])) == [int(x) for x in cur["pivot_idx"]]
        else:
            cur[k] = v


@pytest.mark.parametrize("N,B,seed", [(20000, 16, 1), (100000, 64, 2), (512, 4, 3), (1000, 1, 4),
                                      (33, 7, 5), (4096, 1024, 6), (5000, 3, 7), (17, 17, 8)])
def test_partition_vs_oracle(kd, ctx, oracle_mod, N, B, seed):
    R = synth.rank_like(N, seed)
    if seed == 7:
        R = np.round(R, 2)  # heavy ties
        R[:10] = -0.0
        R[10:20] = 0.0
    say("partition", N, B, seed)
    check_partition_equal(kd, ctx.sample_partition(R, B), oracle_mod.partition(R, B), B)


def test_partition_errors(kd, ctx):
    R = np.zeros(10)
    for B in (0, 11, 2000):
        with pytest.raises(kd.KdError):
            ctx.sample_partition(R, B)


def test_end_to_end_small(kd, ctx, oracle_mod):
    """Count -> rank -> partition on the small workload against the oracle's
    own ranks: buckets identical except within 2x the rank tolerance of a
    pivot."""
    ss = synth.small()
    L = oracle_mod.count(ss)
    R_or, scale = oracle_mod.rank(L, 0.1, with_scale=True)
    p_or = oracle_mod.partition(R_or, ss.B)
    say("end-to-end small")
    kset = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    R = ctx.kmer_rank(kset, 0.1)
    p = ctx.sample_partition(R, ss.B)
    check_ranks(R.cpu().numpy(), R_or, scale)
    bg = kd.u32(p["bucket"])
    diff = np.flatnonzero(bg != p_or["bucket"])
    piv = p_or["pivot_rank"]
    for i in diff:
        assert np.min(np.abs(piv - R_or[i])) <= 2 * RTOL * scale[i], i


# ------------------------------------------------------- full-size sampled

@pytest.mark.parametrize("which", ["paper20k", "large100k"])
def test_full_size_sampled(kd, ctx, oracle_mod, which):
    """The workloads at full size, as bench.py runs them: word lists of every
    sequence bit-exact, sampled rank rows within the tolerance, sampled
    16-row similarity blocks bit-exact, and the split of the GPU's own ranks
    bit-exact against the oracle's split of the same ranks."""
    ss = synth.paper20k() if which == "paper20k" else synth.large100k()
    nrows = 24 if which == "paper20k" else 8
    L = oracle_mod.count(ss)
    say("full-size count", which, ss.n)
    kset = check_lists(kd, ctx, ss, L)
    rng = np.random.default_rng(51)
    rows = np.sort(rng.choice(ss.n, size=nrows, replace=False)).astype(np.uint32)
    say("full-size rank", which)
    R = ctx.kmer_rank(kset, 0.1).cpu().numpy()
    R_or, scale = oracle_mod.rank(L, 0.1, rows=rows, with_scale=True)
    check_ranks(R[rows], R_or, scale)
    say("full-size similarity", which)
    for r0 in (0, ss.n // 2 - 10, ss.n - 16):
        S = kd.u16(ctx.kmer_similarity(kset, r0, 16, 0, ss.n))
        assert np.array_equal(S, oracle_mod.similarity(L, r0, 16, 0, ss.n)[0])
    say("full-size partition", which)
    p = ctx.sample_partition(R, ss.B)
    off = kd.u32(p["offsets"])
    assert off[-1] == ss.n and np.diff(off.astype(np.int64)).max() <= 2 * math.ceil(ss.n / ss.B)
    check_partition_equal(kd, p, oracle_mod.partition(R, ss.B), ss.B)
