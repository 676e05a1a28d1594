"""Pins for the CPU oracle against what the paper and the mathematics fix.

None of these re-type the oracle's code: the k-mer words are checked against
hand-worked values and Python's own base-6 parsing, shared counts against a
dense brute force built through that independent route, ranks against closed
forms and an exactly-rounded sum, and the decomposition against hand-worked
cases and the regular-sampling balance bound of Section 3.2.
"""
import math

import numpy as np
import pytest

import synth
from conftest import golden_lines

AA = "ACDEFGHIKLMNPQRSTVWY"


def _dayhoff():
    return {l.split()[0]: int(l.split()[1]) for l in golden_lines("dayhoff6.txt")}


def _words_indep(seq: str):
    """k-mer words via str.translate + int(text, 6): positional base-6 notation
    is big-endian by definition, independent of the oracle's loop."""
    tab = str.maketrans({k: str(v) for k, v in _dayhoff().items()})
    digits = seq.translate(tab)
    return [int(digits[t:t + 6], 6) for t in range(len(seq) - 5)]


def _dense_indep(seq: str):
    return np.bincount(np.array(_words_indep(seq), dtype=np.int64), minlength=46656)


# ---------------------------------------------------------------- encoding --

def test_dayhoff_groups(oracle_mod):
    g = _dayhoff()
    assert sorted(g) == sorted(AA)
    for ch, v in g.items():
        assert oracle_mod.code(ord(ch)) == v, ch
    for ch in b"BJOUXZacdefg*- \n0":
        assert oracle_mod.code(ch) == -1, chr(ch)


def test_kmer_words_golden(oracle_mod):
    for line in golden_lines("kmer_words.txt"):
        seq, *w = line.split()
        assert list(oracle_mod.kmer_words(seq.encode())) == [int(x) for x in w], seq
        assert _words_indep(seq) == [int(x) for x in w], seq


def test_kmer_words_vs_base6(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(50):
        s = "".join(rng.choice(list(AA), size=int(rng.integers(6, 80))))
        assert list(oracle_mod.kmer_words(s.encode())) == _words_indep(s)


def test_count_errors(oracle_mod):
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.count(synth.from_strings(["ACDEFGH", "ACDXFGH"]))
    assert e.value.code == -2 and e.value.seq == 1 and e.value.pos == 3
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.count(synth.from_strings(["ACDEFGH", "ACDEF"]))
    assert e.value.code == -3 and e.value.seq == 1
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.count(synth.from_strings(["A" * (65535 + 5 + 1)]))
    assert e.value.code == -4
    # the longest allowed sequence: 65535 words
    L = oracle_mod.count(synth.from_strings(["A" * (65535 + 5)]))
    assert L.K[0] == 65535 and list(L.cnt) == [65535]


def test_count_lists_vs_dense(oracle_mod):
    rng = np.random.default_rng(12)
    ss = synth.random_tiny(rng, 24, 6, 120)
    L = oracle_mod.count(ss)
    for i in range(ss.n):
        s = ss.seq(i).decode()
        dense = _dense_indep(s)
        nz = np.flatnonzero(dense)
        ids, cnt = L.entries(i)
        assert np.array_equal(ids, nz)
        assert np.array_equal(cnt, dense[nz])
        assert int(cnt.sum()) == len(s) - 5 == int(L.K[i])
        assert np.all(np.diff(ids.astype(np.int64)) > 0)


# ------------------------------------------------------------ shared count --

@pytest.mark.parametrize("alphabet,seed", [(AA, 1), ("AC", 2), ("ACD", 3), ("AGPSTC", 4)])
def test_shared_vs_dense_bruteforce(oracle_mod, alphabet, seed):
    """Section 3: shared = sum over all epsilon words of min(cX, cY).  Small
    alphabets force repeated words (counts >= 2) so the min matters."""
    rng = np.random.default_rng(seed)
    ss = synth.random_tiny(rng, 20, 6, 90, alphabet.encode())
    L = oracle_mod.count(ss)
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    S, D = oracle_mod.similarity(L, 0, ss.n, 0, ss.n)
    for i in range(ss.n):
        for j in range(ss.n):
            assert S[i, j] == int(np.minimum(dense[i], dense[j]).sum())
            assert D[i, j] == min(len(ss.seq(i)), len(ss.seq(j))) - 5
    # the oracle's literal dense routine agrees too
    cx = oracle_mod.count_dense(ss.seq(0))
    cy = oracle_mod.count_dense(ss.seq(1))
    assert oracle_mod.shared_dense(cx, cy) == S[0, 1]


def test_count_dense_bin_for_bin(oracle_mod):
    """The literal 46,656-bin count vector (the reference for the dense
    export) equals the independent base-6 histogram in every bin, not only
    in its min-sum with another vector."""
    rng = np.random.default_rng(13)
    for alphabet in (AA, "AC", "ACDFHI"):
        for _ in range(6):
            s = "".join(rng.choice(list(alphabet), size=int(rng.integers(6, 300))))
            assert np.array_equal(oracle_mod.count_dense(s.encode()), _dense_indep(s)), s
    s = "A" * (65535 + 5)
    d = oracle_mod.count_dense(s.encode())
    assert d[0] == 65535 and int(d.sum()) == 65535


def test_similarity_offset_blocks_bruteforce(oracle_mod):
    """Section 3 shared counts and Equation 1 denominators on blocks that
    start away from the origin (rows r0.., columns c0..), against the dense
    brute force: a transposed or mis-offset block fails here."""
    rng = np.random.default_rng(14)
    ss = synth.random_tiny(rng, 29, 6, 110, b"ACDEFGH")
    L = oracle_mod.count(ss)
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    n = ss.lengths()
    for r0, nr, c0, nc in ((3, 7, 11, 5), (0, 29, 17, 12), (20, 9, 0, 4), (28, 1, 28, 1), (5, 13, 2, 27)):
        S, D = oracle_mod.similarity(L, r0, nr, c0, nc)
        assert S.shape == (nr, nc)
        for a in range(nr):
            for b in range(nc):
                i, j = r0 + a, c0 + b
                assert S[a, b] == int(np.minimum(dense[i], dense[j]).sum()), (r0, c0, a, b)
                assert D[a, b] == min(n[i], n[j]) - 5


def test_shared_invariants(oracle_mod):
    rng = np.random.default_rng(5)
    ss = synth.random_tiny(rng, 16, 6, 200, b"ACDEFGHIK")
    L = oracle_mod.count(ss)
    S, D = oracle_mod.similarity(L, 0, ss.n, 0, ss.n)
    assert np.array_equal(S, S.T)
    assert np.array_equal(np.diag(S), L.K)
    assert np.all(S <= D)


def test_shared_dayhoff_relabel_metamorphic(oracle_mod):
    """Swapping residues within a Dayhoff group, or renaming the groups
    consistently, leaves every shared count unchanged."""
    rng = np.random.default_rng(6)
    groups = ["AGPST", "C", "DENQ", "FWY", "HKR", "ILMV"]
    ss = synth.random_tiny(rng, 12, 6, 150)
    within = {c: g[int(rng.integers(len(g)))] for g in groups for c in g}
    perm = rng.permutation(6)
    across = {c: groups[perm[k]][0] for k, g in enumerate(groups) for c in g}
    base = oracle_mod.similarity(oracle_mod.count(ss), 0, ss.n, 0, ss.n)[0]
    for m in (within, across):
        t = synth.from_strings(["".join(m[c] for c in ss.seq(i).decode()) for i in range(ss.n)])
        assert np.array_equal(oracle_mod.similarity(oracle_mod.count(t), 0, t.n, 0, t.n)[0], base)


# ------------------------------------------------ fraction, distance, rank --

def test_fraction_distance_closed_forms(oracle_mod):
    for d in (1, 7, 344, 65535):
        assert oracle_mod.fraction(d, d) == 1.0
        assert oracle_mod.fraction(0, d) == 0.0
    for delta in (0.1, 1e-3, 0.5):
        # Delta + 1 is rounded once in double before the log: a relative
        # change of at most 2^-53 in the argument, so at most 2^-53 (1.1e-16)
        # absolute in d; allow that plus one ulp of the log itself.
        assert oracle_mod.distance(1.0, delta) == pytest.approx(-math.log1p(delta), rel=2.3e-16, abs=1.2e-16)
        assert oracle_mod.distance(0.0, delta) == pytest.approx(-math.log(delta), rel=2.3e-16, abs=0)
    # F = 1 - Delta gives distance exactly 0
    assert oracle_mod.distance(0.75, 0.25) == 0.0


def test_rank_worked_example(oracle_mod):
    kv = {}
    for line in golden_lines("worked_rank.txt"):
        k, *v = line.split()
        kv[(k, v[0]) if k == "seq" else k] = v
    delta = float(kv["delta"][0])
    seqs = [kv[("seq", n)][1] for n in "XYZ"]
    L = oracle_mod.count(synth.from_strings(seqs))
    S, D = oracle_mod.similarity(L, 0, 3, 0, 3)
    assert S[0, 1] == int(kv["shared_XY"][0]) and D[0, 1] == int(kv["denom_XY"][0])
    assert S[0, 2] == int(kv["shared_XZ"][0]) and S[1, 2] == int(kv["shared_YZ"][0])
    R = oracle_mod.rank(L, delta)
    # closed forms from Equations 1-3
    rx = (2 * -math.log1p(delta) - math.log(delta)) / 3
    rz = (2 * -math.log(delta) - math.log1p(delta)) / 3
    assert R[0] == R[1]                       # exact tie
    assert R[0] == pytest.approx(rx, rel=1e-15, abs=0)
    assert R[2] == pytest.approx(rz, rel=1e-15, abs=0)
    assert R[0] == pytest.approx(float(kv["rank_X"][0]), rel=1e-15, abs=0)
    assert R[2] == pytest.approx(float(kv["rank_Z"][0]), rel=1e-15, abs=0)


def test_rank_identical_sequences(oracle_mod):
    for delta in (0.1, 0.01):
        L = oracle_mod.count(synth.from_strings(["MKVLAAGIVGLLLAQ"] * 37))
        R = oracle_mod.rank(L, delta)
        np.testing.assert_allclose(R, -math.log1p(delta), rtol=1e-15, atol=0)


def test_rank_disjoint_sequences(oracle_mod):
    """No shared word between any two sequences: R = ((N-1)(-ln D) - ln(1+D))/N."""
    seqs = ["AAAAAAAA", "CCCCCC", "DDDDDDDDDDD", "FFFFFFF", "HHHHHH", "IIIIIIIIIIIIIII",
            "ACACACACAC", "DFDFDFDFDF"]
    L = oracle_mod.count(synth.from_strings(seqs))
    S, _ = oracle_mod.similarity(L, 0, len(seqs), 0, len(seqs))
    assert np.count_nonzero(S - np.diag(np.diag(S))) == 0
    N, delta = len(seqs), 0.1
    expect = ((N - 1) * -math.log(delta) - math.log1p(delta)) / N
    np.testing.assert_allclose(oracle_mod.rank(L, delta), expect, rtol=1e-15, atol=0)


def test_rank_vs_exact_sum_bruteforce(oracle_mod):
    """Equation 3 including the j = i term, summed exactly with math.fsum over
    distances built from the dense brute-force shared counts."""
    rng = np.random.default_rng(7)
    ss = synth.random_tiny(rng, 30, 6, 100, b"ACDEFGHIKLM")
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    n = ss.lengths()
    delta = 0.1
    L = oracle_mod.count(ss)
    R = oracle_mod.rank(L, delta)
    for i in range(ss.n):
        ds = [-math.log(delta + int(np.minimum(dense[i], dense[j]).sum()) / (min(n[i], n[j]) - 5))
              for j in range(ss.n)]
        ref = math.fsum(ds) / ss.n
        assert R[i] == pytest.approx(ref, rel=4e-16, abs=1e-300)


def test_rank_row_subsets_vs_exact_sum(oracle_mod):
    """Equation 3 for a subset of rows (any order, repeats): each row sums
    over all N columns, exactly as for the full set."""
    rng = np.random.default_rng(17)
    ss = synth.random_tiny(rng, 26, 6, 90, b"ACDEFGHIKL")
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    n = ss.lengths()
    delta = 0.07
    L = oracle_mod.count(ss)
    rows = np.array([25, 3, 3, 0, 17, 9], dtype=np.uint32)
    R, sc = oracle_mod.rank(L, delta, rows=rows, with_scale=True)
    assert R.shape == (len(rows),)
    for a, i in enumerate(rows.tolist()):
        ds = [-math.log(delta + int(np.minimum(dense[i], dense[j]).sum()) / (min(n[i], n[j]) - 5))
              for j in range(ss.n)]
        assert R[a] == pytest.approx(math.fsum(ds) / ss.n, rel=4e-16, abs=1e-300)
        assert sc[a] == pytest.approx(math.fsum(abs(d) for d in ds) / ss.n, rel=1e-15)


def test_rank_bounds_and_permutation(oracle_mod):
    s = synth.small()
    sub = synth.from_strings([s.seq(i) for i in range(64)])
    L = oracle_mod.count(sub)
    delta = 0.1
    R = oracle_mod.rank(L, delta)
    assert np.all(R >= -math.log1p(delta) - 1e-15) and np.all(R <= -math.log(delta) + 1e-15)
    perm = np.random.default_rng(8).permutation(64)
    P = oracle_mod.rank(oracle_mod.count(synth.from_strings([sub.seq(int(i)) for i in perm])), delta)
    np.testing.assert_allclose(P, R[perm], rtol=1e-15, atol=0)


# ---------------------------------------------------------- decomposition --

def _cases():
    cur = None
    for line in golden_lines("partition_cases.txt"):
        k, *v = line.split()
        if k == "case":
            cur = {"name": v[0]}
        elif k == "end":
            yield cur
        else:
            cur[k] = v


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c["name"])
def test_partition_golden(oracle_mod, case):
    R = np.array([float(x) for x in case["ranks"]])
    B = int(case["B"][0])
    p = oracle_mod.partition(R, B)
    assert list(p["bucket"]) == [int(x) for x in case["bucket"]]
    assert list(p["offsets"]) == [int(x) for x in case["offsets"]]
    assert list(p["order"]) == [int(x) for x in case["order"]]
    assert list(p["pivot_idx"]) == [int(x) for x in case["pivot_idx"]]
    assert np.array_equal(p["pivot_rank"], R[p["pivot_idx"]])


def _check_partition_invariants(R, B, p):
    N = len(R)
    bucket, order, off = p["bucket"], p["order"], p["offsets"]
    assert sorted(order.tolist()) == list(range(N))
    assert off[0] == 0 and off[-1] == N and np.all(np.diff(off.astype(np.int64)) >= 0)
    assert np.array_equal(np.bincount(bucket, minlength=B), np.diff(off.astype(np.int64)))
    keys = sorted(range(N), key=lambda i: (R[i], i))
    assert list(order) == keys                       # grouped order == key order
    for b in range(B):
        assert np.all(bucket[order[off[b]:off[b + 1]]] == b)
    if N >= B * B:                                   # Section 3.2 bound
        assert np.diff(off.astype(np.int64)).max() <= 2 * math.ceil(N / B)
    assert len(p["pivot_idx"]) == B - 1


@pytest.mark.parametrize("seed", range(30))
def test_partition_invariants_random(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    B = int(rng.integers(1, 13))
    N = int(rng.integers(B, 8 * B * B + 2))
    kind = seed % 4
    if kind == 0:
        R = rng.random(N)
    elif kind == 1:
        R = np.sort(rng.random(N))
    elif kind == 2:
        R = np.sort(rng.random(N))[::-1].copy()
    else:
        R = rng.integers(0, 3, size=N).astype(np.float64)   # heavy ties
    p = oracle_mod.partition(R, B)
    _check_partition_invariants(R, B, p)
    if B == 1:
        assert np.all(p["bucket"] == 0)


def test_partition_errors(oracle_mod):
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.partition(np.zeros(3), 0)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.partition(np.zeros(3), 4)


def test_partition_small_workload(oracle_mod):
    s = synth.small()
    L = oracle_mod.count(s)
    R = oracle_mod.rank(L, 0.1)
    p = oracle_mod.partition(R, s.B)
    _check_partition_invariants(R, s.B, p)


# ------------------------------------------------------ globalized rank --

def _global_cases():
    cases, cur = [], None
    for line in golden_lines("worked_global_rank.txt"):
        k, *v = line.split()
        if k == "case":
            cur = {"name": v[0]}
            cases.append(cur)
        else:
            cur[k] = v
    return cases


@pytest.mark.parametrize("case", _global_cases(), ids=lambda c: c["name"])
def test_global_rank_worked(oracle_mod, case):
    delta = 0.1
    L1, L0 = -math.log1p(delta), -math.log(delta)
    val = {"L1": L1, "L0": L0, "H": (L1 + L0) / 2}
    ss = synth.from_strings(case["seqs"])
    L = oracle_mod.count(ss)
    B, k = int(case["B"][0]), int(case["k"][0])
    loc = oracle_mod.local_ranks(L, B, delta)
    smp = oracle_mod.global_samples(loc, B, k)
    assert smp.tolist() == [int(x) for x in case["samples"]]
    G = oracle_mod.global_rank(L, smp, delta)
    np.testing.assert_allclose(G, [val[x] for x in case["global"]], rtol=1e-15, atol=0)


def _block_bounds(N, B):
    return [(b * N // B, (b + 1) * N // B) for b in range(B)]


def test_local_ranks_vs_exact_sum_bruteforce(oracle_mod):
    """Steps 1-2: Equation 3 over each block alone, summed exactly."""
    rng = np.random.default_rng(21)
    ss = synth.random_tiny(rng, 23, 6, 90, b"ACDEFGHIKL")
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    n = ss.lengths()
    delta = 0.05
    L = oracle_mod.count(ss)
    for B in (1, 2, 3, 5):
        loc = oracle_mod.local_ranks(L, B, delta)
        for lo, hi in _block_bounds(ss.n, B):
            for i in range(lo, hi):
                ds = [-math.log(delta + int(np.minimum(dense[i], dense[j]).sum()) / (min(n[i], n[j]) - 5))
                      for j in range(lo, hi)]
                assert loc[i] == pytest.approx(math.fsum(ds) / (hi - lo), rel=4e-16, abs=1e-300)


def test_local_ranks_special_cases(oracle_mod):
    """One block is the centralized rank; each block equals the centralized
    rank of that block taken on its own."""
    s = synth.small()
    sub = synth.from_strings([s.seq(i) for i in range(70)])
    L = oracle_mod.count(sub)
    delta = 0.1
    np.testing.assert_array_equal(oracle_mod.local_ranks(L, 1, delta), oracle_mod.rank(L, delta))
    loc = oracle_mod.local_ranks(L, 4, delta)
    for lo, hi in _block_bounds(70, 4):
        part = oracle_mod.count(synth.from_strings([sub.seq(i) for i in range(lo, hi)]))
        np.testing.assert_array_equal(loc[lo:hi], oracle_mod.rank(part, delta))


def test_global_samples_rule(oracle_mod):
    """Steps 3-5 against an independent selection: sort each block by (rank,
    index) with Python's sort and take positions floor(t w / (k+1))."""
    rng = np.random.default_rng(5)
    for N, B, k in ((40, 3, 2), (97, 8, 7), (64, 4, 16), (10, 10, 1), (33, 2, 16)):
        R = np.round(rng.random(N) * 8) / 8  # many ties, broken by index
        smp = oracle_mod.global_samples(R, B, k)
        want = []
        for lo, hi in _block_bounds(N, B):
            order = sorted(range(lo, hi), key=lambda i: (R[i], i))
            want += [order[t * (hi - lo) // (k + 1)] for t in range(1, k + 1)]
        assert smp.tolist() == want
    # k = w_b takes every sequence of the block once
    R = rng.random(60)
    smp = oracle_mod.global_samples(R, 4, 15)
    assert sorted(smp.tolist()) == list(range(60))
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.global_samples(R, 4, 16)   # k above a block's size
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.global_samples(R, 4, 0)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.global_samples(R, 61, 1)


def test_global_rank_vs_exact_sum_bruteforce(oracle_mod):
    """Step 6: Equation 3 with the gathered samples as the set (a sample is
    one of its own terms), summed exactly."""
    rng = np.random.default_rng(22)
    ss = synth.random_tiny(rng, 31, 6, 80, b"ACDEFGHIKLMN")
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    n = ss.lengths()
    delta = 0.1
    L = oracle_mod.count(ss)
    smp = np.array([3, 17, 17, 0, 30, 9], dtype=np.uint32)   # any list, repeats allowed
    G, sc = oracle_mod.global_rank(L, smp, delta, with_scale=True)
    for i in range(ss.n):
        ds = [-math.log(delta + int(np.minimum(dense[i], dense[j]).sum()) / (min(n[i], n[j]) - 5))
              for j in smp.tolist()]
        assert G[i] == pytest.approx(math.fsum(ds) / len(ds), rel=4e-16, abs=1e-300)
        assert sc[i] == pytest.approx(math.fsum(abs(d) for d in ds) / len(ds), rel=1e-15)


def test_global_rank_row_subsets_vs_exact_sum(oracle_mod):
    """Step 6 for a subset of rows: the same samples, summed exactly."""
    rng = np.random.default_rng(23)
    ss = synth.random_tiny(rng, 27, 6, 85, b"ACDEFGHIKLMN")
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    n = ss.lengths()
    delta = 0.1
    L = oracle_mod.count(ss)
    smp = np.array([4, 26, 11, 11, 0], dtype=np.uint32)
    rows = np.array([26, 0, 13, 13, 5], dtype=np.uint32)
    G, sc = oracle_mod.global_rank(L, smp, delta, rows=rows, with_scale=True)
    for a, i in enumerate(rows.tolist()):
        ds = [-math.log(delta + int(np.minimum(dense[i], dense[j]).sum()) / (min(n[i], n[j]) - 5))
              for j in smp.tolist()]
        assert G[a] == pytest.approx(math.fsum(ds) / len(ds), rel=4e-16, abs=1e-300)
        assert sc[a] == pytest.approx(math.fsum(abs(d) for d in ds) / len(ds), rel=1e-15)


def test_global_rank_all_sampled_is_centralized(oracle_mod):
    """With k = w_b every sequence is a sample, so the globalized rank is the
    centralized rank (Equation 3) up to summation order."""
    s = synth.small()
    sub = synth.from_strings([s.seq(i) for i in range(96)])
    L = oracle_mod.count(sub)
    delta = 0.1
    for B in (1, 3, 8):
        loc = oracle_mod.local_ranks(L, B, delta)
        smp = oracle_mod.global_samples(loc, B, 96 // B)
        G = oracle_mod.global_rank(L, smp, delta)
        np.testing.assert_allclose(G, oracle_mod.rank(L, delta), rtol=2e-15, atol=0)


# ------------------------------------------- per-bucket matrices and trees --

def test_upgma_worked(oracle_mod):
    n = 5
    d = np.zeros((n, n))
    want = []
    for line in golden_lines("worked_upgma.txt"):
        k, *v = line.split()
        if k == "d":
            i, j, x = int(v[0]), int(v[1]), float(v[2])
            d[i, j] = d[j, i] = x
        else:
            want.append((int(v[0]), int(v[1]), float(v[2])))
    m, h = oracle_mod.upgma(d)
    assert [tuple(x) for x in m.tolist()] == [w[:2] for w in want]
    assert h.tolist() == [w[2] for w in want]


def test_upgma_all_equal_ties(oracle_mod):
    """Every distance 1: ties go to the lowest slots, so the cluster in slot
    0 absorbs the leaves in index order."""
    n = 6
    m, h = oracle_mod.upgma(np.ones((n, n)))
    assert m.tolist() == [[0, 1], [2, 6], [3, 7], [4, 8], [5, 9]]
    assert h.tolist() == [0.5] * 5


def _lca_height_matrix(rng, n):
    """A random ultrametric: random binary merges of leaves with distinct
    integer heights; D[i][j] = 2 x height of the lowest common ancestor."""
    clusters = [[i] for i in range(n)]
    D = np.zeros((n, n))
    merges = []
    for step, hgt in enumerate(range(1, n)):
        a, b = sorted(rng.choice(len(clusters), size=2, replace=False))
        A, Bc = clusters[a], clusters[b]
        for i in A:
            for j in Bc:
                D[i, j] = D[j, i] = 2.0 * hgt
        merges.append((frozenset(A), frozenset(Bc), float(hgt)))
        clusters = [c for q, c in enumerate(clusters) if q not in (a, b)] + [A + Bc]
    return D, merges


def test_upgma_recovers_ultrametric(oracle_mod):
    """On an ultrametric matrix UPGMA returns its tree: the same clusters
    merge at half their LCA distance (integer heights keep every average
    exact)."""
    rng = np.random.default_rng(3)
    for n in (2, 3, 9, 25):
        D, tree = _lca_height_matrix(rng, n)
        m, h = oracle_mod.upgma(D)
        members = {i: frozenset([i]) for i in range(n)}
        got = []
        for t, (x, y) in enumerate(m.tolist()):
            members[n + t] = members[x] | members[y]
            got.append((frozenset([members[x], members[y]]), h[t]))
        want = [(frozenset([A, Bc]), hgt) for A, Bc, hgt in tree]
        assert sorted(got, key=lambda g: g[1]) == sorted(want, key=lambda g: g[1])


def _upgma_by_leaf_means(d):
    """Independent average linkage: the distance of two clusters is the mean
    of the original distances over all leaf pairs across them (no update
    formula); ties by the clusters' smallest leaves."""
    n = d.shape[0]
    clusters = {i: [i] for i in range(n)}
    out = []
    for t in range(n - 1):
        best = None
        keys = sorted(clusters, key=lambda c: min(clusters[c]))
        for ia, a in enumerate(keys):
            for b in keys[ia + 1:]:
                v = math.fsum(d[i, j] for i in clusters[a] for j in clusters[b]) / (
                    len(clusters[a]) * len(clusters[b]))
                if best is None or v < best[0]:
                    best = (v, a, b)
        v, a, b = best
        out.append((min(a, b), max(a, b), v / 2))
        clusters[n + t] = clusters.pop(a) + clusters.pop(b)
    return out


def test_upgma_vs_leaf_means(oracle_mod):
    rng = np.random.default_rng(11)
    for n in (2, 4, 7, 12):
        x = rng.random((n, n))
        d = (x + x.T) / 2
        m, h = oracle_mod.upgma(d)
        want = _upgma_by_leaf_means(d)
        assert [tuple(r) for r in m.tolist()] == [w[:2] for w in want]
        np.testing.assert_allclose(h, [w[2] for w in want], rtol=1e-13, atol=0)
        assert np.all(np.diff(h) >= 0)   # average linkage merges at non-decreasing heights


def test_upgma_errors_and_one_leaf(oracle_mod):
    m, h = oracle_mod.upgma(np.zeros((1, 1)))
    assert m.shape == (0, 2) and h.shape == (0,)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.upgma(np.zeros((0, 0)))


def test_distance_matrix_bruteforce(oracle_mod):
    """Equations 1-2 from dense brute-force counts, any subset and order of
    sequences; the diagonal is -ln(1 + Delta)."""
    rng = np.random.default_rng(13)
    ss = synth.random_tiny(rng, 17, 6, 70, b"ACDEFGHIK")
    dense = [_dense_indep(ss.seq(i).decode()) for i in range(ss.n)]
    n = ss.lengths()
    L = oracle_mod.count(ss)
    idx = np.array([5, 0, 16, 3, 3, 9], dtype=np.uint32)
    delta = 0.07
    M = oracle_mod.distance_matrix(L, idx, delta)
    for r, i in enumerate(idx):
        for c, j in enumerate(idx):
            s = int(np.minimum(dense[i], dense[j]).sum())
            want = -math.log(delta + s / (min(n[i], n[j]) - 5))
            assert M[r, c] == pytest.approx(want, rel=1e-15, abs=1e-300)
    np.testing.assert_allclose(np.diag(M), -math.log1p(delta), rtol=1e-15, atol=0)
    np.testing.assert_array_equal(M, M.T)


# --------------------------------------------------- profiles and PSP (Eq. 4) --

def _joint(rng):
    """A symmetric joint distribution of aligned amino-acid pairs."""
    x = rng.random((20, 20)) + 0.05
    P = x + x.T
    return P / P.sum()


def test_profile_worked(oracle_mod):
    """Three rows: column 0 = A, A, C -> A 2/3, C 1/3; column 1 = -, G, G ->
    G 2/3 (one gap); column 2 = W, ., - -> W 1/3; column 3 = Y, Y, Y."""
    aln = np.frombuffer(b"A-WY" b"AG.Y" b"CG-Y", dtype=np.uint8).reshape(3, 4)
    f = oracle_mod.profile(aln)
    idx = {chr(c): i for i, c in enumerate(oracle_mod.AMINO)}
    want = np.zeros((4, 20))
    want[0, idx["A"]] = 2 / 3
    want[0, idx["C"]] = 1 / 3
    want[1, idx["G"]] = 2 / 3
    want[2, idx["W"]] = 1 / 3
    want[3, idx["Y"]] = 1.0
    np.testing.assert_allclose(f, want, rtol=1e-15, atol=0)
    assert oracle_mod.AMINO == b"".join(sorted(oracle_mod.AMINO[i:i + 1] for i in range(20)))
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.profile(np.frombuffer(b"AB-", dtype=np.uint8).reshape(1, 3))
    assert e.value.pos == 1


def test_psp_one_hot_and_bilinear(oracle_mod):
    """A column holding only amino acid i against one holding only j scores
    M[i][j]; the score is linear in each column's frequencies."""
    rng = np.random.default_rng(17)
    M = oracle_mod.psp_matrix(_joint(rng))
    E = np.eye(20)
    np.testing.assert_allclose(oracle_mod.psp(E, E, M), M, rtol=1e-15, atol=1e-15)
    fx = rng.random((3, 20))
    fy = rng.random((4, 20))
    S = oracle_mod.psp(fx, fy, M)
    for x in range(3):
        for y in range(4):
            terms = [fx[x, i] * fy[y, j] * M[i, j] for i in range(20) for j in range(20)]
            assert S[x, y] == pytest.approx(math.fsum(terms), rel=1e-13, abs=1e-13)
    a, b = rng.random(2)
    mix = oracle_mod.psp(a * fx[:1] + b * fx[1:2], fy, M)
    np.testing.assert_allclose(mix, a * S[:1] + b * S[1:2], rtol=1e-12, atol=1e-13)
    # symmetric M: swapping the profiles transposes the scores
    np.testing.assert_allclose(oracle_mod.psp(fy, fx, M), S.T, rtol=1e-13, atol=1e-14)


def test_psp_matrix_definition(oracle_mod):
    """Independent pairs (P = p p^T) give log 1 = 0 everywhere; doubling one
    diagonal weight and renormalising gives a closed form."""
    p = np.arange(1, 21, dtype=np.float64)
    p /= p.sum()
    np.testing.assert_allclose(oracle_mod.psp_matrix(np.outer(p, p)), 0.0, atol=1e-13)
    P = np.full((20, 20), 1.0)
    P[0, 0] = 2.0
    P /= P.sum()           # p_0 = 21/401, others 20/401
    M = oracle_mod.psp_matrix(P)
    assert M[0, 0] == pytest.approx(math.log((2 / 401) / (21 / 401) ** 2), rel=1e-14)
    assert M[1, 2] == pytest.approx(math.log((1 / 401) / (20 / 401) ** 2), rel=1e-14)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.psp_matrix(np.zeros((20, 20)))
