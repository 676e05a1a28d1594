"""GPU: the step after the split -- the buckets' sequences gathered, each
bucket's k-mer distance matrix (Equations 1-2) and its UPGMA guide tree --
through the C ABI against the oracle.

Bars: gathered residues and offsets bit-exact; distances within 1e-12
relative (1e-14 absolute near zero) of the oracle; UPGMA merges and heights
bit-exact against the oracle's UPGMA of the same matrix (both sides take
every merge decision on the same numbers with the same arithmetic)."""
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_1744_amd as kd
    kd.lib()
    return kd


@pytest.fixture(scope="module")
def ctx(kd):
    c = kd.Context()
    yield c
    c.synchronize()


def split_mats(D, first):
    D = D.cpu().numpy()
    out, o = [], 0
    for a, b in zip(first[:-1], first[1:]):
        n = int(b) - int(a)
        out.append(D[o:o + n * n].reshape(n, n))
        o += n * n
    return out


def close(G, O):
    np.testing.assert_allclose(G, O, rtol=1e-12, atol=1e-14)


def gpu_tree(ctx, kd, mats):
    first = np.concatenate([[0], np.cumsum([m.shape[0] for m in mats])]).astype(np.uint32)
    flat = np.concatenate([m.ravel() for m in mats])
    m, h = ctx.upgma(first, flat)
    m, h = m.cpu().numpy(), h.cpu().numpy()
    out, o = [], 0
    for mat in mats:
        k = mat.shape[0] - 1
        out.append((m[o:o + k], h[o:o + k]))
        o += k
    return out


def test_gather_matches_numpy(kd, ctx):
    rng = np.random.default_rng(61)
    ss = synth.random_tiny(rng, 90, 6, 300)
    off = ss.offsets.astype(np.int64)
    for order in (rng.permutation(ss.n), rng.choice(ss.n, size=40, replace=False), np.array([], np.int64),
                  np.array([3, 3, 7, 0])):
        say("gather", len(order))
        res, o = ctx.gather_sequences(ss.residues, off, order.astype(np.int32))
        want = b"".join(ss.seq(int(i)) for i in order)
        lens = [len(ss.seq(int(i))) for i in order]
        assert np.array_equal(o.cpu().numpy(), np.concatenate([[0], np.cumsum(lens)]).astype(np.int64))
        assert res.cpu().numpy()[:len(want)].tobytes() == want


def test_gather_errors(kd, ctx):
    ss = synth.from_strings(["ACDEFGHIK", "LMNPQRSTVW", "AAAAAAAAAAAAAAAAAAAA"])
    off = ss.offsets.astype(np.int64)
    with pytest.raises(kd.KdError):
        ctx.gather_sequences(ss.residues, off, np.array([0, 3], np.int32))   # index out of range
    with pytest.raises(kd.KdError):  # more residues than the output holds
        ctx.gather_sequences(ss.residues, off, np.array([2, 2, 2], np.int32))


def test_distance_matrices_vs_oracle(kd, ctx, oracle_mod):
    rng = np.random.default_rng(62)
    sets = [synth.random_tiny(rng, n, 6, 400) for n in (1, 2, 17, 64, 65, 130)] + synth.batched(9, 3)
    res, off, first, _ = synth.concat(sets)
    say("distances", [x.n for x in sets])
    kb = ctx.kmer_count_batch(res, off.view(np.int64), first)
    for delta in (0.1, 0.003):
        mats = split_mats(ctx.distance_matrices(kb, delta), first)
        for x, M in zip(sets, mats):
            L = oracle_mod.count(x)
            O = oracle_mod.distance_matrix(L, np.arange(x.n), delta)
            close(M, O)
            assert np.array_equal(M, M.T)
    kb.destroy()


def _ultrametric(rng, n):
    clusters = [[i] for i in range(n)]
    D = np.zeros((n, n))
    tree = []
    for hgt in range(1, n):
        a, b = sorted(rng.choice(len(clusters), size=2, replace=False))
        A, Bc = clusters[a], clusters[b]
        D[np.ix_(A, Bc)] = 2.0 * hgt
        D[np.ix_(Bc, A)] = 2.0 * hgt
        tree.append((frozenset([frozenset(A), frozenset(Bc)]), float(hgt)))
        clusters = [c for q, c in enumerate(clusters) if q not in (a, b)] + [A + Bc]
    return D, tree


def _hubs(rng, n, hubs):
    """Every row before hub column c has its minimum there (value v plus a
    little noise): merging two hubs leaves hundreds of rows to rescan at
    once, more than the merge kernel has waves."""
    x = rng.random((n, n)) + 2.0
    for c, v in hubs:
        x[:c, c] = v + rng.random(c) * 1e-3
    x = np.triu(x, 1)
    return x + x.T


def test_upgma_given_matrices(kd, ctx, oracle_mod):
    rng = np.random.default_rng(63)
    mats = []
    for n in (1, 2, 3, 9, 50, 301):
        x = rng.random((n, n))
        mats.append((x + x.T) / 2)
    mats.append(np.ones((7, 7)))                        # every pair ties
    q = np.round(rng.random((40, 40)) * 4) / 4          # many ties
    mats.append(np.triu(q) + np.triu(q, 1).T)
    w = np.zeros((5, 5))
    for (i, j), v in {(0, 1): 2, (0, 2): 6, (0, 3): 10, (0, 4): 9, (1, 2): 6, (1, 3): 10, (1, 4): 9,
                      (2, 3): 10, (2, 4): 9, (3, 4): 8}.items():
        w[i, j] = w[j, i] = v
    mats.append(w)                                      # the worked example
    mats.append(_ultrametric(rng, 64)[0])
    mats.append(_hubs(rng, 200, [(150, 0.5), (151, 0.6), (160, 0.1)]))
    mats.append(_hubs(rng, 1500, [(900, 0.2), (901, 0.21), (1400, 0.3), (1401, 0.31)]))  # two rows per thread
    say("upgma", [m.shape[0] for m in mats])
    for mat, (m, h) in zip(mats, gpu_tree(ctx, kd, mats)):
        om, oh = oracle_mod.upgma(mat)
        assert np.array_equal(m, om), mat.shape
        assert np.array_equal(h, oh), mat.shape
    assert gpu_tree(ctx, kd, [w])[0][1].tolist() == [1.0, 3.0, 4.0, 4.75]


def test_upgma_largest_set(kd, ctx):
    """4096 members (the largest accepted) on an ultrametric matrix: the
    tree comes back exactly; 4097 is refused."""
    rng = np.random.default_rng(64)
    D, tree = _ultrametric(rng, 4096)
    say("upgma 4096")
    (m, h), = gpu_tree(ctx, kd, [D])
    members = {i: frozenset([i]) for i in range(4096)}
    got = []
    for t, (x, y) in enumerate(m.tolist()):
        members[4096 + t] = members[x] | members[y]
        got.append((frozenset([members[x], members[y]]), h[t]))
    assert sorted(got, key=lambda g: g[1]) == sorted(tree, key=lambda g: g[1])
    with pytest.raises(kd.KdError):
        gpu_tree(ctx, kd, [np.zeros((4097, 4097))])


def test_upgma_errors(kd, ctx):
    bad = np.zeros((4, 4))
    bad[1, 2] = bad[2, 1] = float("nan")
    bad[0, :] = bad[:, 0] = float("nan")
    bad[3, :] = bad[:, 3] = float("nan")
    with pytest.raises(kd.KdError):
        gpu_tree(ctx, kd, [bad])
    with pytest.raises(ValueError):
        ctx.upgma(np.array([0, 3], np.uint32), np.zeros(8))


def check_bucket_trees(kd, ctx, oracle_mod, ss, R, B, full_buckets):
    out = ctx.bucket_trees(ss.residues, ss.offsets.view(np.int64), R, B)
    first = out["set_first"]
    order = kd.u32(out["order"])
    mats = split_mats(out["dist"], first)
    m_all, h_all = out["merges"].cpu().numpy(), out["heights"].cpu().numpy()
    L = oracle_mod.count(ss)
    rng = np.random.default_rng(65)
    o = 0
    for b in range(B):
        a, e = int(first[b]), int(first[b + 1])
        n = e - a
        idx = order[a:e]
        M = mats[b]
        m, h = m_all[o:o + n - 1], h_all[o:o + n - 1]
        o += n - 1
        if b in full_buckets:
            close(M, oracle_mod.distance_matrix(L, idx, 0.1))
            om, oh = oracle_mod.upgma(M)
            assert np.array_equal(m, om) and np.array_equal(h, oh), b
        else:
            rows = rng.choice(n, size=min(n, 4), replace=False)
            close(M[rows], oracle_mod.distance_block(L, idx[rows], idx, 0.1))
        assert np.all(np.diff(h) >= 0)                 # average linkage is monotone
        ids = m.ravel()
        assert sorted(ids.tolist()) == list(range(2 * n - 2))  # every node merged once


def test_bucket_trees_small(kd, ctx, oracle_mod):
    ss = synth.small()
    ks = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    R = ctx.kmer_rank(ks, 0.1)
    say("bucket trees small", ss.n, ss.B)
    check_bucket_trees(kd, ctx, oracle_mod, ss, R, ss.B, full_buckets=range(ss.B))


def test_bucket_trees_paper20k(kd, ctx, oracle_mod):
    """Full size (20,000 sequences, 16 buckets of about 1,250): one bucket
    checked whole against the oracle, the others on sampled rows and tree
    invariants."""
    ss = synth.paper20k()
    ks = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    R = ctx.kmer_rank(ks, 0.1)
    say("bucket trees 20k")
    check_bucket_trees(kd, ctx, oracle_mod, ss, R, ss.B, full_buckets=[7])


def test_distance_matrices_large_set(kd, ctx, oracle_mod):
    """A set larger than the permutation's LDS row (4,096) beside a small
    one: sampled rows against the oracle (all columns), symmetry and the
    diagonal everywhere."""
    rng = np.random.default_rng(64)
    big = synth.from_strings([synth.small(5).seq(i % 512) + b"ACDEFGHIKLMNPQRSTVWY"[i % 20:i % 20 + 3] * (1 + i % 3)
                              for i in range(4200)])
    sets = [big, synth.random_tiny(rng, 70, 6, 300)]
    res, off, first, _ = synth.concat(sets)
    say("distances large", [x.n for x in sets])
    kb = ctx.kmer_count_batch(res, off.view(np.int64), first)
    mats = split_mats(ctx.distance_matrices(kb, 0.1), first)
    kb.destroy()
    M = mats[0]
    L = oracle_mod.count(big)
    rows = np.unique(np.concatenate([[0, 1, 4095, 4096, 4199], rng.integers(0, big.n, 27)]))
    close(M[rows], oracle_mod.distance_block(L, rows, np.arange(big.n), 0.1))
    assert np.array_equal(M, M.T)
    close(np.diag(M), np.full(big.n, -np.log(1.1)))
    close(mats[1], oracle_mod.distance_matrix(oracle_mod.count(sets[1]), np.arange(70), 0.1))
