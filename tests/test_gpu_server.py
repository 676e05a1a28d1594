"""GPU: the request server.  Every served job's results must match the CPU
oracle (ranks within 1e-12 of the tolerance scale, Equation 3; the split
bit-exact on the served ranks and, against the oracle's own ranks, identical
except next to a pivot, Section 3.1.2) and be bit-identical to the same job
run alone through the single-set calls; admission must keep the reserved
bytes within the budget; bad jobs fail alone; cancellation of queued jobs;
one-job-at-a-time mode."""
import concurrent.futures as cf
import os
import sys
import time

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


@pytest.fixture(scope="module")
def jobs():
    ss = np.random.SeedSequence(77).spawn(16)
    out = [synth.served_job(s, 64, 1500) for s in ss]
    rng = np.random.default_rng(8)
    out.append(synth.random_tiny(rng, 3, 6, 40))   # B = 1
    out.append(synth.random_tiny(rng, 70, 6, 90))
    return out


@pytest.fixture(scope="module")
def oracle_jobs():
    """Served-shape jobs (the served workload's generator: N log-uniform,
    B = max(1, N/256)) for the oracle comparison, one of them with N > 4096
    and B = 16 so that its split runs on the large-workgroup radix path."""
    ss = np.random.SeedSequence(91).spawn(6)
    out = [synth.served_job(ss[0], 4200, 4400)]
    out += [synth.served_job(s, 64, 1400) for s in ss[1:]]
    rng = np.random.default_rng(9)
    out.append(synth.random_tiny(rng, 5, 6, 50))
    return out


def oracle_rank(oracle, L, delta):
    """Equation 3 for every row, the rows split over host threads (the
    oracle's C runs outside the interpreter lock); returns ranks, scale."""
    n = L.n
    nt = max(1, min(16, os.cpu_count() or 1))
    chunks = [np.arange(a, min(n, a + 64), dtype=np.uint32) for a in range(0, n, 64)]
    with cf.ThreadPoolExecutor(nt) as ex:
        parts = list(ex.map(lambda r: oracle.rank(L, delta, rows=r, with_scale=True), chunks))
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


@pytest.fixture(scope="module")
def oracle_results(oracle_mod, oracle_jobs):
    out = []
    for q, x in enumerate(oracle_jobs):
        delta = 0.1 if q % 2 == 0 else 0.05
        L = oracle_mod.count(x)
        R, scale = oracle_rank(oracle_mod, L, delta)
        out.append(dict(delta=delta, R=R, scale=scale, part=oracle_mod.partition(R, x.B)))
    return out


@pytest.mark.parametrize("mirror", [True, False], ids=["device-copies", "host-copies"])
def test_server_matches_oracle(kd, oracle_mod, oracle_jobs, oracle_results, mirror):
    """Every served job against the CPU oracle: ranks within 1e-12 x the
    scale (1/N) sum_j |d(i,j)|; the split of the served ranks bit-exact
    against the oracle's split of those same ranks; buckets against the
    oracle's own split identical except for a rank within twice the
    tolerance of a pivot."""
    srv = kd.Server(0, device_mirror=mirror)
    say("server-oracle", [x.n for x in oracle_jobs], "mirror", mirror)
    tickets = [(srv.submit(x.residues, x.offsets, x.B, oracle_results[q]["delta"]), q)
               for q, x in enumerate(oracle_jobs)]
    recs = drain(srv, len(tickets), timeout=120.0)
    assert any(recs[t]["batch_jobs"] > 1 for t, _ in tickets)
    for t, q in tickets:
        x, want, rec = oracle_jobs[q], oracle_results[q], recs[t]
        assert rec["status"] == 0, (q, rec["status"])
        err = np.abs(rec["ranks"] - want["R"]) / want["scale"]
        assert float(err.max()) <= 1e-12, (q, x.n, float(err.max()))
        own = oracle_mod.partition(rec["ranks"], x.B)
        for k in ("bucket", "order", "offsets"):
            assert np.array_equal(rec[k], own[k]), (q, k)
        pr = want["part"]
        diff = np.flatnonzero(rec["bucket"] != pr["bucket"])
        for i in diff:
            gap = np.min(np.abs(pr["pivot_rank"] - want["R"][i]))
            assert gap <= 2e-12 * want["scale"][i], (q, int(i), gap)
        if diff.size == 0:
            assert np.array_equal(rec["offsets"], pr["offsets"]), q
        # the served order is the oracle's key order up to near-ties (ranks
        # within twice the tolerance may swap, e.g. exactly tied ranks)
        Ro = want["R"][rec["order"].astype(np.int64)]
        so = want["scale"][rec["order"].astype(np.int64)]
        assert np.all(Ro[:-1] <= Ro[1:] + 2e-12 * np.maximum(so[:-1], so[1:])), q
        assert x.B == max(1, x.n // 256)
    srv.close()


def alone(ctx, kd, x, delta):
    ks = ctx.kmer_count(x.residues, x.offsets.view(np.int64))
    R = ctx.kmer_rank(ks, delta)
    p = ctx.sample_partition(R, x.B)
    return dict(ranks=R.cpu().numpy(), bucket=kd.u32(p["bucket"]), order=kd.u32(p["order"]),
                offsets=kd.u32(p["offsets"]))


def drain(srv, n, timeout=60.0):
    recs, t0 = [], time.monotonic()
    while len(recs) < n:
        recs += srv.poll(64, wait_s=0.05)
        assert time.monotonic() - t0 < timeout, f"only {len(recs)} of {n} records"
    return {r["ticket"]: r for r in recs}


def check_same(rec, want):
    assert rec["status"] == 0, rec["status"]
    for k in ("ranks", "bucket", "order", "offsets"):
        assert np.array_equal(rec[k], want[k]), k


@pytest.mark.parametrize("mirror", [True, False], ids=["device-copies", "host-copies"])
def test_server_matches_alone(kd, ctx, jobs, mirror):
    """Batches gather their input from the jobs' device copies (sent at
    submit) or, without mirrors, send it from the host copies."""
    srv = kd.Server(0, device_mirror=mirror)
    say("server", len(jobs), "mirror", mirror)
    tickets = []
    for q, x in enumerate(jobs):
        delta = 0.1 if q % 3 else 0.05
        tickets.append((srv.submit(x.residues, x.offsets, x.B, delta), q, delta))
    recs = drain(srv, len(tickets))
    batched = 0
    for t, q, delta in tickets:
        check_same(recs[t], alone(ctx, kd, jobs[q], delta))
        assert recs[t]["t_submit_ns"] <= recs[t]["t_start_ns"] <= recs[t]["t_done_ns"]
        batched += recs[t]["batch_jobs"] > 1
    assert batched > 0  # jobs submitted together share batches
    srv.close()


@pytest.mark.parametrize("mirror", [True, False], ids=["device-copies", "host-copies"])
def test_server_bad_job_fails_alone(kd, ctx, jobs, mirror):
    srv = kd.Server(0, device_mirror=mirror)
    bad = jobs[1].residues.copy()
    bad[int(jobs[1].offsets[5]) + 2] = ord("B")
    short = synth.from_strings(["ACDEFGH", "ACD"])
    t0 = srv.submit(jobs[0].residues, jobs[0].offsets, jobs[0].B)
    t1 = srv.submit(bad, jobs[1].offsets, jobs[1].B)
    t2 = srv.submit(short.residues, short.offsets, 1)
    t3 = srv.submit(jobs[2].residues, jobs[2].offsets, jobs[2].B)
    recs = drain(srv, 4)
    assert recs[t1]["status"] == -2
    assert recs[t2]["status"] == -3
    check_same(recs[t0], alone(ctx, kd, jobs[0], 0.1))
    check_same(recs[t3], alone(ctx, kd, jobs[2], 0.1))
    with pytest.raises(kd.KdError):  # inconsistent offsets are refused at submit
        srv.submit(jobs[0].residues[:-1], jobs[0].offsets, jobs[0].B)
    with pytest.raises(kd.KdError):
        srv.submit(jobs[0].residues, jobs[0].offsets, jobs[0].n + 1)
    srv.close()


def test_server_budget_and_fifo(kd, ctx, jobs):
    sizes = [kd.job_bytes(x.residues.size, x.n) for x in jobs]
    budget = 2 * max(sizes)
    srv = kd.Server(0, hbm_budget=budget)
    say("server-budget", budget)
    with pytest.raises(kd.KdError) as e:  # a job that can never fit
        big = synth.served_job(np.random.SeedSequence(5), 4000, 4000)
        srv2 = kd.Server(0, hbm_budget=kd.job_bytes(big.residues.size, big.n) - 1)
        try:
            srv2.submit(big.residues, big.offsets, big.B)
        finally:
            srv2.close()
    assert e.value.status == -6
    tickets = [(srv.submit(x.residues, x.offsets, x.B), q) for q, x in enumerate(jobs)]
    peak = 0
    recs = {}
    t0 = time.monotonic()
    while len(recs) < len(tickets):
        st = srv.status()
        assert st["reserved"] <= budget
        peak = max(peak, st["reserved"])
        for r in srv.poll(64, wait_s=0.01):
            recs[r["ticket"]] = r
        assert time.monotonic() - t0 < 60
    assert srv.status()["reserved"] == 0
    for t, q in tickets:
        check_same(recs[t], alone(ctx, kd, jobs[q], 0.1))
    srv.close()
    # one job at a time
    srv = kd.Server(0, max_batch_jobs=1)
    tickets = [(srv.submit(x.residues, x.offsets, x.B), q) for q, x in enumerate(jobs[:6])]
    recs = drain(srv, len(tickets))
    for t, q in tickets:
        assert recs[t]["batch_jobs"] == 1
        check_same(recs[t], alone(ctx, kd, jobs[q], 0.1))
    srv.close()


def test_server_cancel(kd, ctx, jobs):
    # budget for one job: the rest queue, so cancelling the last is possible
    srv = kd.Server(0, hbm_budget=max(kd.job_bytes(x.residues.size, x.n) for x in jobs[:4]))
    ts = [srv.submit(x.residues, x.offsets, x.B) for x in jobs[:4]]
    rc = srv.cancel(ts[-1])
    assert rc in (0, -6)  # KD_EBUSY only if it already started
    assert srv.cancel(10 ** 9) == -1
    recs = drain(srv, 4)
    if rc == 0:
        assert recs[ts[-1]]["status"] == -8
    for q, t in enumerate(ts[:3]):
        check_same(recs[t], alone(ctx, kd, jobs[q], 0.1))
    srv.close()


def overlap_ms(tl):
    """Device time during which a batch's stage A (count, layout) ran while
    the previous batch's stage B (rank, split, copy back) was running."""
    tot = 0.0
    for prev, cur in zip(tl, tl[1:]):
        a0, a1 = cur["count"]
        b0, b1 = prev["rank"]
        tot += max(0.0, min(a1, b1) - max(a0, b0))
    return tot


def test_server_pipeline_timeline(kd, ctx, jobs):
    """Batches of at most 4 jobs through the two stages: every job is
    bit-identical to running it alone, each batch's stages are ordered on the
    device (its stage B starts after its stage A ends), and the records
    report how much of each stage A ran during the previous stage B."""
    srv = kd.Server(0, max_batch_jobs=4, timeline=True)
    say("server-pipeline", len(jobs))
    tickets = [(srv.submit(x.residues, x.offsets, x.B), q) for q, x in enumerate(jobs)]
    recs = drain(srv, len(tickets))
    for t, q in tickets:
        check_same(recs[t], alone(ctx, kd, jobs[q], 0.1))
    tl = srv.timeline()
    assert len(tl) >= (len(jobs) + 3) // 4 - 1 and sum(b["jobs"] for b in tl) <= len(jobs)
    for b in tl:
        assert b["count"][0] <= b["count"][1] <= b["rank"][0] <= b["rank"][1]
    for prev, cur in zip(tl, tl[1:]):
        assert prev["rank"][0] <= cur["rank"][0]
    say("stage A overlapping stage B: %.3f ms over %d batches" % (overlap_ms(tl), len(tl)))
    srv.close()


def test_server_mirrors_within_budget(kd, ctx, jobs):
    """The input mirrors count against the budget: with room for them, the
    reserved bytes (jobs + mirrors) never pass the budget during a burst and
    every job still matches running it alone."""
    sizes = [kd.job_bytes(x.residues.size, x.n) for x in jobs]
    budget = (64 << 20) * 2 + 2 * max(sizes)   # one mirror chunk fits (half the budget)
    srv = kd.Server(0, hbm_budget=budget, max_batch_jobs=3)
    tickets = [(srv.submit(x.residues, x.offsets, x.B), q) for q, x in enumerate(jobs) for _ in range(2)]
    recs, t0 = {}, time.monotonic()
    while len(recs) < len(tickets):
        assert srv.status()["reserved"] <= budget
        for r in srv.poll(64, wait_s=0.005):
            recs[r["ticket"]] = r
        assert time.monotonic() - t0 < 60
    assert srv.status()["reserved"] <= 64 << 20  # the mirror stays; the jobs' charges are gone
    for t, q in tickets:
        check_same(recs[t], alone(ctx, kd, jobs[q], 0.1))
    srv.close()
