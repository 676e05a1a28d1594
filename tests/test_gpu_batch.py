"""GPU: the batched calls (many independent sets per call) against the
single-set calls on each set alone and against the CPU oracle.

Bars: per set, ranks, buckets, order and offsets bit-identical to what the
single-set calls give for that set (the rank accumulation is exact and each
set keeps its own tiling); word lists bit-exact; ranks of small sets within
the oracle tolerance; splits of given rank arrays identical to the oracle's.
"""
import dataclasses
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
    kd.lib()
    return kd


@pytest.fixture(scope="module")
def ctx(kd):
    c = kd.Context()
    yield c
    c.synchronize()


def as_set(res, off, name="batch"):
    return synth.SeqSet(res, off, np.zeros(off.size - 1, np.int32), name, 1)


def mixed_sets():
    """Sizes around every tile boundary (16-row blocks, 64-column groups,
    32-group strips), tiny sets, and sets drawn like the batched workload."""
    rng = np.random.default_rng(41)
    out = []
    for n, B in [(1, 1), (2, 2), (5, 3), (16, 4), (17, 1), (63, 7), (64, 8), (65, 2), (77, 5),
                 (300, 8), (1000, 31), (2100, 16)]:
        x = synth.random_tiny(rng, n, 6, 400)
        out.append(dataclasses.replace(x, B=B))
    out += synth.batched(4, 12)
    perm = rng.permutation(len(out))
    return [out[i] for i in perm]


def single(ctx, kd, x, delta):
    ks = ctx.kmer_count(x.residues, x.offsets.view(np.int64))
    R = ctx.kmer_rank(ks, delta)
    p = ctx.sample_partition(R, x.B)
    return (R.cpu().numpy(), kd.u32(p["bucket"]), kd.u32(p["order"]), kd.u32(p["offsets"]))


def split_batch(kd, out, first, Bs):
    R = out["ranks"].cpu().numpy()
    bucket, order, offs = kd.u32(out["bucket"]), kd.u32(out["order"]), kd.u32(out["offsets"])
    ob = np.concatenate([[0], np.cumsum(Bs.astype(np.int64) + 1)])
    for q in range(len(Bs)):
        a, b = int(first[q]), int(first[q + 1])
        yield R[a:b], bucket[a:b], order[a:b], offs[ob[q]:ob[q + 1]]


@pytest.mark.parametrize("delta", [0.1, 1e-3])
def test_batch_matches_single(kd, ctx, delta):
    sets = mixed_sets()
    res, off, first, Bs = synth.concat(sets)
    say("batch-vs-single", len(sets), int(first[-1]), delta)
    out = ctx.batch_run(res, off.view(np.int64), first, Bs, delta)
    for q, got in enumerate(split_batch(kd, out, first, Bs)):
        want = single(ctx, kd, sets[q], delta)
        for name, g, w in zip(("ranks", "bucket", "order", "offsets"), got, want):
            assert np.array_equal(g, w), (q, sets[q].n, name)


def test_batch_lists_and_ranks_vs_oracle(kd, ctx, oracle_mod):
    sets = [s for s in mixed_sets() if s.n <= 400]
    res, off, first, Bs = synth.concat(sets)
    say("batch-lists", len(sets), int(first[-1]))
    ks = ctx.kmer_count_batch(res, off.view(np.int64), first)
    assert ks.nsets == len(sets) and ks.n == int(first[-1])
    ids, cnt, eoff = ks.export_lists()
    L = oracle_mod.count(as_set(res, off))
    assert np.array_equal(eoff.cpu().numpy().astype(np.uint64), L.off)
    assert np.array_equal(kd.u16(ids), L.ids)
    assert np.array_equal(kd.u16(cnt), L.cnt)
    R = ctx.kmer_rank(ks, 0.1).cpu().numpy()
    for q, x in enumerate(sets):
        a, b = int(first[q]), int(first[q + 1])
        R_or, scale = oracle_mod.rank(oracle_mod.count(x), 0.1, with_scale=True)
        err = np.abs(R[a:b] - R_or)
        assert (err <= RTOL * scale).all(), (q, x.n, err.max())


@pytest.mark.parametrize("cases", [
    [(20000, 16), (4096, 1024), (33, 7), (1, 1), (17, 17), (1000, 1), (5000, 3), (777, 8)],
    # every set at most 4,096 keys and samples: the small-workgroup kernel
    [(4096, 64), (33, 7), (1, 1), (17, 17), (1000, 1), (2000, 3), (777, 8), (4000, 40), (64, 64)],
], ids=["large-sets", "small-sets"])
def test_partition_batch_vs_oracle(kd, ctx, oracle_mod, cases):
    Rs = []
    for q, (n, B) in enumerate(cases):
        R = synth.rank_like(n, 100 + q)
        if q == 6:
            R = np.round(R, 2)
            R[:10] = -0.0
            R[10:20] = 0.0
        Rs.append(R)
    first = np.concatenate([[0], np.cumsum([n for n, _ in cases])]).astype(np.uint32)
    Bs = np.array([B for _, B in cases], dtype=np.uint32)
    say("partition-batch", len(cases))
    p = ctx.sample_partition_batch(np.concatenate(Rs), first, Bs)
    bucket, order, offs = kd.u32(p["bucket"]), kd.u32(p["order"]), kd.u32(p["offsets"])
    pidx, prank = kd.u32(p["pivot_idx"]), p["pivot_rank"].cpu().numpy()
    ob, pb = 0, 0
    for q, (n, B) in enumerate(cases):
        a, b = int(first[q]), int(first[q + 1])
        want = oracle_mod.partition(Rs[q], B)
        assert np.array_equal(bucket[a:b], want["bucket"]), q
        assert np.array_equal(order[a:b], want["order"]), q
        assert np.array_equal(offs[ob:ob + B + 1], want["offsets"]), q
        assert np.array_equal(pidx[pb:pb + B - 1], want["pivot_idx"]), q
        assert np.array_equal(prank[pb:pb + B - 1], want["pivot_rank"]), q
        ob += B + 1
        pb += B - 1


def test_batch_errors(kd, ctx):
    rng = np.random.default_rng(5)
    sets = [synth.random_tiny(rng, n, 6, 50) for n in (10, 20, 30)]
    res, off, first, Bs = synth.concat(sets)
    bad = res.copy()
    bad[int(off[first[1] + 4]) + 3] = ord("X")  # set 1, sequence 4, position 3
    with pytest.raises(kd.KdError) as e:
        ctx.kmer_count_batch(bad, off.view(np.int64), first)
    assert e.value.status == -2 and e.value.seq == int(first[1]) + 4 and e.value.pos == 3
    with pytest.raises(kd.KdError):
        ctx.kmer_count_batch(res, off.view(np.int64), np.array([0, 20, 10, 60], np.uint32))
    with pytest.raises(kd.KdError):
        ctx.kmer_count_batch(res, off.view(np.int64), np.array([1, 10, 30, 60], np.uint32))
    with pytest.raises(ValueError):  # bounds must end at the number of sequences
        ctx.kmer_count_batch(res, off.view(np.int64), np.array([0, 10, 30, 61], np.uint32))
    with pytest.raises(kd.KdError):
        ctx.batch_run(res, off.view(np.int64), first, np.array([1, 21, 1], np.uint32))
    with pytest.raises(kd.KdError):
        ctx.batch_run(res, off.view(np.int64), first, np.array([1, 0, 1], np.uint32))
    ks = ctx.kmer_count_batch(res, off.view(np.int64), first)
    with pytest.raises(kd.KdError):
        ctx.kmer_similarity(ks, 0, 2, 0, 2)
    # empty sets inside a batch count as nothing
    first_e = np.array([0, 0, 10, 10, 30, 60, 60], np.uint32)
    ks2 = ctx.kmer_count_batch(res, off.view(np.int64), first_e)
    R2 = ctx.kmer_rank(ks2, 0.1).cpu().numpy()
    R1 = ctx.kmer_rank(ks, 0.1).cpu().numpy()
    assert np.array_equal(R1, R2)


def test_batched_workload_sampled(kd, ctx, oracle_mod):
    """512 sets drawn like the batched workload, run as one batch; 32
    sampled sets against the single-set calls, 3 small ones against the
    oracle."""
    sets = synth.batched(4, 512)
    res, off, first, Bs = synth.concat(sets)
    say("batched-512", int(first[-1]))
    out = ctx.batch_run(res, off.view(np.int64), first, Bs, 0.1)
    parts = list(split_batch(kd, out, first, Bs))
    rng = np.random.default_rng(3)
    for q in rng.choice(len(sets), 32, replace=False):
        want = single(ctx, kd, sets[q], 0.1)
        for name, g, w in zip(("ranks", "bucket", "order", "offsets"), parts[q], want):
            assert np.array_equal(g, w), (q, sets[q].n, name)
    small = [q for q in range(len(sets)) if sets[q].n <= 80][:3]
    for q in small:
        R_or, scale = oracle_mod.rank(oracle_mod.count(sets[q]), 0.1, with_scale=True)
        assert (np.abs(parts[q][0] - R_or) <= RTOL * scale).all(), q


def test_autotune_shapes_identical(kd, ctx):
    """Every work-list shape gives bit-identical ranks; the tuned shape is
    used by later counts of the same size class (single set and batch)."""
    import torch
    ss = synth.paper20k(2, 3000)
    say("autotune", ss.n)
    ks = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
    R0 = ctx.kmer_rank(ks, 0.1).clone()
    best, ms = ctx.autotune(ks, 0.1)
    assert best in ctx.TUNE_SHAPES and all(v > 0 for v in ms.values())
    # the fewest tasks within 1% of the fastest
    fastest = min(ms.values())
    assert ms[best] <= fastest * 1.01
    assert all(ms[t] > fastest * 1.01 for t in ctx.TUNE_SHAPES if t < best)
    assert torch.equal(ctx.kmer_rank(ks, 0.1), R0)
    for t in (1, 3, 64):  # any shape, set by hand, gives the same ranks
        ctx.set_tasks_per_cu(1, ss.n, t)
        ks2 = ctx.kmer_count(ss.residues, ss.offsets.view(np.int64))
        assert torch.equal(ctx.kmer_rank(ks2, 0.1), R0), t
    sets = synth.batched(4, 40)
    res, off, first, Bs = synth.concat(sets)
    kb = ctx.kmer_count_batch(res, off.view(np.int64), first)
    Rb = ctx.kmer_rank(kb, 0.1).clone()
    best, _ = ctx.autotune(kb, 0.1)
    kb2 = ctx.kmer_count_batch(res, off.view(np.int64), first)
    assert torch.equal(ctx.kmer_rank(kb2, 0.1), Rb)


def test_batch_plan_graph_replays(kd, ctx):
    """The batch captured as one HIP graph (kd_batch_plan): every replay, with
    eager work and synchronizations between replays, writes the eager
    kd_batch_run outputs again bit for bit."""
    import torch
    sets = synth.batched(4, 60)
    res, off, first, Bs = synth.concat(sets)
    say("batch plan", len(sets), "sets", int(first[-1]), "sequences")
    want = {k: v.clone() for k, v in ctx.batch_run(res, off.view(np.int64), first, Bs, 0.1).items()}
    plan = ctx.batch_plan(res, off.view(np.int64), first, Bs, 0.1)
    assert plan.launches >= 8
    other = synth.paper20k(9, 700)
    for rep in range(3):
        for k, t in plan.out.items():
            t.fill_(-1)
        plan.launch()
        ks = ctx.kmer_count(other.residues, other.offsets.view(np.int64))  # eager work in between
        ctx.kmer_rank(ks, 0.1)
        ks.destroy()
        ctx.synchronize()
        for k, w in want.items():
            g = plan.out[k][:w.numel()]
            if k == "ranks":
                g, w = g.view(torch.int64), w.view(torch.int64)
            assert torch.equal(g, w), (rep, k)
    plan.destroy()
