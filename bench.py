#!/usr/bin/env python3
"""Benchmark: one step = k-mer counting -> all-pairs similarity + k-mer rank
-> regular-sampling split, on the paper-scale synthetic workload (N = 20,000
protein sequences in 200 families, Dayhoff-6 k = 6, B = 16 buckets,
delta = 0.1), inputs resident in HBM before timing starts.

Prints one JSON line with the whole-job throughput in k-mer pair
similarities per second, the roofline position of the dominant kernel (the
all-pairs rank kernel, timed live with HIP events on its stream), and the
single-threaded CPU oracle timed on a bounded sample of the same job.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-mer pair-similarities/sec (GPU vs oracle); p50/p99 request latency"
# MI355X: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 VALU lane-instructions/s; a
# probe (one 16-bit min + add of the shared-count sum) is counted at one
# lane-instruction, i.e. the packed-int16 rate of 78.6e12 ops/s / 2.
PEAK_TPROBE = 256 * 64 * 2.4e9 / 1e12

WORKLOADS = {
    "paper20k": ("paper-scale: N=20000 sequences, 200 families, lognormal length mean 350, "
                 "divergence 5-30%, Dayhoff-6 k=6, B=16, delta=0.1, seed 2"),
    "small": "small: N=512, 8 families, length U[200,400], divergence 10%, B=4, delta=0.1, seed 1",
    "large100k": ("large: N=100000, 1000 families, lognormal mean 300, divergence 5-40%, "
                  "B=64, delta=0.1, seed 3"),
}


# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by
# a plain-copy calibration (profiles/rank_pairs_paper20k.md, rank_pairs_large100k.md,
# profiles/rank_cross_global100k.md).  Reported only while the kernel's
# sources hash to the measured version and the same work-list shape is in use.
RANK_SOURCES = ["paper_0905_1744_amd/csrc/pair.hip", "paper_0905_1744_amd/csrc/tile.h",
                "paper_0905_1744_amd/csrc/bitcount.h", "paper_0905_1744_amd/csrc/klog.h"]
BATCH_SOURCES = RANK_SOURCES + ["paper_0905_1744_amd/csrc/worklist.h"]  # the batch's work-list order
TREE_SOURCES = ["paper_0905_1744_amd/csrc/tree.hip", "paper_0905_1744_amd/csrc/tile.h",
                "paper_0905_1744_amd/csrc/bitcount.h", "paper_0905_1744_amd/csrc/klog.h",
                "paper_0905_1744_amd/csrc/radix.h"]
TRAFFIC = {
    # key: (kernel, workload).  bytes_per_launch: one number, or for the rank
    # kernel a dict keyed by the work-list shape (tasks per compute unit) the
    # counters were taken at
    ("rank_pairs_kernel", "paper20k"): {"sources": RANK_SOURCES, "sha256_16": "0ebbc92f3c550ca3",
                                        "bytes_per_launch": {16: 209310720, 32: 204222805, 64: 253211392,
                                                             128: 251519403}},
    ("rank_pairs_kernel", "large100k"): {"sources": RANK_SOURCES, "sha256_16": "0ebbc92f3c550ca3",
                                         "bytes_per_launch": {32: 6209227435, 64: 4580742827, 128: 4033544832}},
    ("rank_cross_kernel", "global100k"): {"sources": ["paper_0905_1744_amd/csrc/cross.hip",
                                                      "paper_0905_1744_amd/csrc/tile.h",
                                                      "paper_0905_1744_amd/csrc/bitcount.h",
                                                      "paper_0905_1744_amd/csrc/klog.h"],
                                          "sha256_16": "a24f7da4dc1db0fa",
                                          "bytes_per_launch": 2042262869},
    ("dist_pairs_kernel", "trees20k"): {"sources": TREE_SOURCES, "sha256_16": "d11a4ff3326eb917",
                                        "bytes_per_launch": 571903424},
    ("upgma_kernel", "trees20k"): {"sources": TREE_SOURCES, "sha256_16": "d11a4ff3326eb917",
                                   "bytes_per_launch": 1006388171},
    # the 4,096-set batch's one rank launch (profiles/batched_4096sets.md)
    ("rank_pairs_kernel", "batched"): {"sources": BATCH_SOURCES, "sha256_16": "7ed972ae344349a1",
                                       "bytes_per_launch": {64: 2631491243}},
    # psp_g_kernel + psp_scores_kernel, the two launches of one psp_scores call
    ("psp", "psp"): {"sources": ["paper_0905_1744_amd/csrc/psp.hip"], "sha256_16": "27c995852957b595",
                     "bytes_per_launch": 94294016 + 2873273344},
}


# Unit occupancy of the rank kernel from rocprofv3 SQ counters (the 20k
# profile: SQ_INSTS_VALU, SQ_LDS_IDX_ACTIVE and SQ_LDS_BANK_CONFLICT per
# compute unit over GRBM_GUI_ACTIVE cycles per XCC), reported while the
# kernel's sources hash to the profiled version.
COUNTERS = {
    ("rank_pairs_kernel", "paper20k"): {"sources": RANK_SOURCES, "sha256_16": "0ebbc92f3c550ca3",
                                        "valu_busy": 0.56, "lds_busy": 0.61,
                                        "lds_bank_conflict_share_of_lds_busy": 0.63,
                                        "source": "profiles/rank_pairs_paper20k.md"},
    ("rank_pairs_kernel", "batched"): {"sources": BATCH_SOURCES, "sha256_16": "7ed972ae344349a1",
                                       "tasks_per_cu": 64, "valu_busy": 0.40, "lds_busy": 0.37,
                                       "lds_bank_conflict_share_of_lds_busy": 0.59,
                                       "source": "profiles/batched_4096sets.md"},
}


def profiled_counters(kernel, workload):
    c = COUNTERS.get((kernel, workload))
    if c is None or sources_hash(c["sources"]) != c["sha256_16"]:
        return None
    return {k: v for k, v in c.items() if k not in ("sources", "sha256_16")}


def sources_hash(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, shape):
    t = TRAFFIC.get((kernel, workload))
    if t is None or sources_hash(t["sources"]) != t["sha256_16"]:
        return None
    b = t["bytes_per_launch"]
    return b.get(shape) if isinstance(b, dict) else b


def probe_count(D):
    """sum over unordered pairs of min(D_i, D_j) (work of walking the shorter list)."""
    import numpy as np
    d = np.sort(np.asarray(D, dtype=np.int64))
    n = d.shape[0]
    return int((d * (n - 1 - np.arange(n))).sum())


def cpu_baseline(ss, delta, budget_s):
    """Time the CPU oracle (single thread) on the first M rows of the rank
    (each row is N pair similarities) and extrapolate the whole job."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    L = oracle.count(ss)
    t_count = time.perf_counter() - t0
    N = ss.n
    rows = np.arange(min(8, N), dtype=np.uint32)
    t0 = time.perf_counter()
    oracle.rank(L, delta, rows=rows)
    per_row = (time.perf_counter() - t0) / len(rows)
    M = int(min(N, max(len(rows), budget_s / max(per_row, 1e-9))))
    rows = np.arange(M, dtype=np.uint32)
    t0 = time.perf_counter()
    oracle.rank(L, delta, rows=rows)
    t_rows = time.perf_counter() - t0
    job_s = t_count + t_rows * N / M
    pairs = N * (N - 1) / 2
    return {
        "value": pairs / job_s,
        "unit": "pair-similarities/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle k-mer counting of all {N} sequences ({t_count:.2f} s) + rank rows "
                   f"0..{M - 1} each against all {N} sequences ({t_rows:.2f} s, {M * N} pair "
                   f"similarities), single thread; job time extrapolated to all {N} rows = "
                   f"{job_s:.1f} s"),
    }


def cpu_baseline_all_cores(ss, delta, budget_s, L=None):
    """The same oracle on every core the run may use: rows dealt round-robin
    to P threads (ctypes releases the GIL during the oracle's C calls, so the
    threads run in parallel), timed on the wall clock and extrapolated to the
    whole job like the single-thread leg."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    nproc = os.cpu_count() or 1
    P = max(1, min(nproc, int(os.environ.get("KD_CPU_THREADS", "16"))))
    t0 = time.perf_counter()
    if L is None:
        L = oracle.count(ss)
    t_count = time.perf_counter() - t0
    N = ss.n
    probe = np.arange(min(8, N), dtype=np.uint32)
    t0 = time.perf_counter()
    oracle.rank(L, delta, rows=probe)
    per_row = (time.perf_counter() - t0) / len(probe)
    M = int(min(N, max(P, P * budget_s / max(per_row, 1e-9))))
    chunks = [np.arange(p, M, P, dtype=np.uint32) for p in range(P)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=P) as ex:
        list(ex.map(lambda r: oracle.rank(L, delta, rows=r), chunks))
    t_rows = time.perf_counter() - t0
    job_s = t_count + t_rows * N / M
    pairs = N * (N - 1) / 2
    return {
        "value": pairs / job_s,
        "unit": "pair-similarities/s",
        "cores": P,
        "host_nproc": nproc,
        "kind": "oracle",
        "sample": (f"oracle k-mer counting of all {N} sequences (one thread, {t_count:.2f} s) + rank "
                   f"rows 0..{M - 1} against all {N} sequences on {P} threads ({t_rows:.2f} s wall, "
                   f"{M * N} pair similarities); job time extrapolated to all {N} rows = {job_s:.1f} s"),
    }


def group_lengths(D):
    """Padded list length of every column group of one set: group g holds
    the 64 consecutive sequences g*64 .. g*64+63 in ascending-D order and
    its lanes walk max D rounded up to 16 words."""
    import numpy as np
    d = np.sort(np.asarray(D, dtype=np.int64))
    n = d.size
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    g = np.arange((n + 63) // 64)
    return (d[np.minimum(64 * g + 63, n - 1)] + 15) // 16 * 16


def rank_lookups(D):
    """64-lane LDS mask lookups of one all-pairs launch over one set (the
    rank kernel, the distance kernel): column group g walks its padded list
    once against each of the 16-row blocks rb >= 4g."""
    import numpy as np
    L = group_lengths(D)
    RB = (len(D) + 15) // 16
    return int((L * np.maximum(RB - 4 * np.arange(L.size), 0)).sum())


def cross_lookups(D, first, S):
    """Lookups of the globalized rank's cross pass: every column group of
    every block walks its padded list once against each 16-row block of the
    S gathered samples."""
    return int(sum(int(group_lengths(D[a:b]).sum()) for a, b in zip(first[:-1], first[1:]))) * ((S + 15) // 16)


def rank_roofline(probes, pairs, lookups, t_kernel, ceiling, traffic, alg_bytes, kernel="rank_pairs_kernel",
                  counters=None):
    """Roofline of an all-pairs rank launch.  The kernel is bound by its LDS
    mask lookups: one 64-lane random 16-bit read of the row block's table
    answers 16 rows x 64 columns of (word, pair) probes.  achieved = the
    algorithmic probes sum_{i<j} min(D_i, D_j) per second; peak = the
    lookup ceiling measured on this device (kd_calibrate_lds, random reads)
    times the 1,024 probe slots of a lookup."""
    peak = ceiling * 1024 / 1e12
    achieved = probes / t_kernel / 1e12
    return {"bound": "lds", "achieved": achieved, "peak": peak, "unit": "Tprobe/s",
            "frac": achieved / peak, "traffic": traffic, "kernel": kernel, "kernel_ms": t_kernel * 1e3,
            "work_per_launch": {"probes": probes, "pairs": pairs, "wave_lds_lookups": lookups,
                                "probe_slots_used": probes / (lookups * 1024.0),
                                "algorithmic_bytes": alg_bytes},
            "peak_note": ("no published rate exists for random 16-bit LDS reads: the peak is the rate "
                          "kd_calibrate_lds measures live (random indices, 32 reads in flight per lane; "
                          "bank conflicts hold it near 8 CU-cycles per 64-lane read), times 16 rows x 64 "
                          "columns per lookup; conflict-free reads at the published 128 B/clk/CU would "
                          "allow 8x that"),
            "lookups": {"achieved": lookups / t_kernel, "peak": ceiling, "unit": "64-lane reads/s",
                        "frac": lookups / t_kernel / ceiling},
            "probe_per_lane_cycle": {"achieved": achieved, "peak": PEAK_TPROBE,
                                     "ratio": achieved / PEAK_TPROBE,
                                     "note": "the probes against one per VALU lane-cycle (256 CUs x 64 lanes x 2.4 GHz)"},
            "hbm": {"bytes_per_launch": traffic, "frac": (traffic / t_kernel / 8e12) if traffic else None,
                    "algorithmic_bytes": alg_bytes},
            "unit_occupancy_from_counters": counters}


def lds_ceiling(ctx, workgroups=1024, steps=64):
    """Measured rate of random 16-bit LDS reads (32 in flight per lane) over
    the whole chip, in 64-lane reads per second (kd_calibrate_lds)."""
    ctx.calibrate_lds(workgroups, 4, 32)  # warm-up
    ms, n = ctx.calibrate_lds(workgroups, steps, 32)
    return n / (ms / 1e3)


def probe_count_cross(D, smp):
    """sum over (sequence, sample) pairs of min(D_i, D_s)."""
    import numpy as np
    d = np.sort(np.asarray(D, dtype=np.int64))
    ds = np.asarray(D, dtype=np.int64)[np.asarray(smp, dtype=np.int64)]
    c = np.concatenate([[0], np.cumsum(d)])
    k = np.searchsorted(d, ds, side="right")            # sequences with D_i <= D_s
    return int((c[k] + ds * (d.size - k)).sum())


def table1(Rc, G, bc, bg):
    """The statistics of the paper's Table 1 (centralized against globalized
    ranks) plus how many sequences both splits put in the same bucket."""
    import numpy as np
    diff = G - Rc
    rc = np.argsort(np.argsort(Rc, kind="stable"), kind="stable").astype(np.float64)
    rg = np.argsort(np.argsort(G, kind="stable"), kind="stable").astype(np.float64)
    return {"centralized_max": float(Rc.max()), "centralized_min": float(Rc.min()),
            "centralized_mean": float(Rc.mean()), "globalized_max": float(G.max()),
            "globalized_min": float(G.min()), "globalized_mean": float(G.mean()),
            "variance_wrt_centralized": float((diff ** 2).mean()),
            "std_wrt_centralized": float(math.sqrt((diff ** 2).mean())),
            "spearman": float(np.corrcoef(rc, rg)[0, 1]),
            "same_bucket_frac": float((bc == bg).mean())}


def bench_global(args):
    """Algorithm 2 steps 1-11 on one device with the globalized rank: count
    the B blocks as a batch, rank each block against itself, pick k = B - 1
    samples per block, rank every sequence against the k*B samples, split."""
    import numpy as np
    import torch

    import paper_0905_1744_amd as kd
    import synth

    which = {"global20k": "paper20k", "global100k": "large100k"}[args.workload]
    ss = synth.paper20k() if which == "paper20k" else synth.large100k()
    N, B, delta = ss.n, ss.B, args.delta
    k = B - 1
    print(f"[bench] globalized rank on {which}: N={N} B={B} k={k}", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    res = torch.from_numpy(ss.residues).to(dev)
    off = torch.from_numpy(ss.offsets.view(np.int64)).to(dev)
    ctx = kd.Context(0)
    loc = torch.empty(N, dtype=torch.float64, device=dev)
    G = torch.empty(N, dtype=torch.float64, device=dev)

    def step():
        kb = ctx.kmer_count_blocks(res, off, B)
        ctx.kmer_rank(kb, delta, out=loc)
        _, smp = ctx.kmer_rank_global(kb, loc, k, delta, out=G)
        part = ctx.sample_partition(G, B)
        return kb, smp, part

    tune = None
    for w in range(args.warmup):
        kb, smp, _ = step()
        if w == 0 and not args.no_autotune:
            best, ms = ctx.autotune(kb, delta)
            tune = {"tasks_per_cu": best, "ms_per_shape": ms}
        kb.destroy()
    ctx.enable_timing(True, stages=("pairs", "global"))
    ctx.reset_timing()
    kb = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if kb is not None:
            kb.destroy()
        kb, smp, part = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ctx.stage_times()
    nb = min(args.steps, 5)
    ctx.enable_timing(True)
    ctx.reset_timing()
    for _ in range(nb):
        kb.destroy()
        kb, smp, part = step()
    stages = ctx.stage_times()
    ctx.enable_timing(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    first = kb.set_first()  # the library's Algorithm 2 step 1 blocks
    w = np.diff(first.astype(np.int64))
    local_pairs = int((w * (w - 1) // 2).sum())
    cross_pairs = N * k * B
    value = (local_pairs + cross_pairs) / (ms_per_step / 1e3)
    _, _, loff = kb.export_lists()
    D = np.diff(loff.cpu().numpy())
    probes_local = sum(probe_count(D[a:b]) for a, b in zip(first[:-1], first[1:]))
    probes_cross = probe_count_cross(D, kd.u32(smp))
    t_loc = st["pairs"][0] / max(st["pairs"][1], 1) / 1e3
    t_cross = st["global"][0] / max(st["global"][1], 1) / 1e3
    bounds = list(zip(first[:-1], first[1:]))
    lookups_local = sum(rank_lookups(D[a:b]) for a, b in bounds if b > a)
    lookups_cross = cross_lookups(D, first, int(len(smp)))
    ceiling = lds_ceiling(ctx)

    # the comparison of the paper's Table 1, outside the timed region
    kc = ctx.kmer_count(res, off)
    Rc = ctx.kmer_rank(kc, delta)
    pc = ctx.sample_partition(Rc, B)
    cmp = table1(Rc.cpu().numpy(), G.cpu().numpy(), kd.u32(pc["bucket"]), kd.u32(part["bucket"]))
    kc.destroy()
    line = {
        "metric": METRIC, "value": value, "unit": "pair-similarities/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16/f64",
        "data": "synthetic",
        "config": {"workload": "globalized rank, " + WORKLOADS[which], "N": N, "B": B, "k": k,
                   "delta": delta, "pairs_per_step": {"local": local_pairs, "cross": cross_pairs},
                   "step": ("kmer_count_batch (B blocks) + kmer_rank (local ranks) + "
                            "kmer_rank_global + sample_partition"), "autotune": tune},
        "stages_ms_per_step": {k_: v[0] / nb for k_, v in stages.items() if v[1]},
        "roofline": rank_roofline(probes_local, local_pairs, lookups_local, t_loc, ceiling, None,
                                  int(D.sum()) * 2 + 8 * N, kernel="rank_pairs_kernel (local ranks)"),
        "roofline_cross": rank_roofline(probes_cross, cross_pairs, lookups_cross, t_cross, ceiling,
                                        measured_traffic("rank_cross_kernel", args.workload, None),
                                        int(D.sum()) * 2 + 8 * N, kernel="rank_cross_kernel"),
        "table1": cmp,
    }
    kb.destroy()
    ctx.close()
    print(json.dumps(line), flush=True)


def bench_trees(args):
    """The step after the split (Section 3.1.3's input): the B buckets'
    sequences gathered, each bucket's k-mer distance matrix and its UPGMA
    guide tree.  The ranks come from the centralized rank, computed before
    the timed region."""
    import numpy as np
    import torch

    import paper_0905_1744_amd as kd
    import synth

    which = {"trees20k": "paper20k", "trees100k": "large100k"}[args.workload]
    ss = synth.paper20k() if which == "paper20k" else synth.large100k()
    N, B, delta = ss.n, ss.B, args.delta
    print(f"[bench] bucket guide trees on {which}: N={N} B={B}", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    res = torch.from_numpy(ss.residues).to(dev)
    off = torch.from_numpy(ss.offsets.view(np.int64)).to(dev)
    ctx = kd.Context(0)
    ks = ctx.kmer_count(res, off)
    R = ctx.kmer_rank(ks, delta)
    ks.destroy()

    def step():
        return ctx.bucket_trees(res, off, R, B, delta)

    for _ in range(args.warmup):
        out = step()
    torch.cuda.synchronize()
    ctx.enable_timing(True, stages=("dist", "tree"))
    ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ctx.stage_times()
    nb = min(args.steps, 3)
    ctx.enable_timing(True)
    ctx.reset_timing()
    for _ in range(nb):
        out = step()
    stages = ctx.stage_times()
    ctx.enable_timing(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    first = out["set_first"].astype(np.int64)
    n = np.diff(first)
    pairs = int((n * (n - 1) // 2).sum())
    t_dist = st["dist"][0] / max(st["dist"][1], 1) / 1e3
    t_tree = st["tree"][0] / max(st["tree"][1], 1) / 1e3
    # the bucket matrices' pairs: lists of both sequences; work = sum of min(D)
    kb = ctx.kmer_count_batch(*ctx.gather_sequences(res, off, out["order"]), first.astype(np.uint32))
    _, _, loff = kb.export_lists()
    D = np.diff(loff.cpu().numpy())
    kb.destroy()
    probes = sum(probe_count(D[a:b]) for a, b in zip(first[:-1], first[1:]))
    lookups = sum(rank_lookups(D[a:b]) for a, b in zip(first[:-1], first[1:]) if b > a)
    ceiling = lds_ceiling(ctx)
    line = {
        "metric": METRIC, "value": pairs / (ms_per_step / 1e3), "unit": "pair-similarities/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16/f64",
        "data": "synthetic",
        "config": {"workload": "bucket guide trees, " + WORKLOADS[which], "N": N, "B": B, "delta": delta,
                   "bucket_sizes": {"min": int(n.min()), "max": int(n.max())}, "pairs_per_step": pairs,
                   "step": ("sample_partition + kd_gather_sequences + kmer_count_batch (buckets) + "
                            "kmer_distance_matrices + upgma_trees")},
        "stages_ms_per_step": {k: v[0] / nb for k, v in stages.items() if v[1]},
        "roofline": rank_roofline(probes, pairs, lookups, t_dist, ceiling,
                                  measured_traffic("dist_pairs_kernel", args.workload, None),
                                  int(D.sum()) * 2 + 8 * pairs, kernel="dist_pairs_kernel"),
        "upgma": {"kernel": "upgma_kernel", "ms": t_tree * 1e3, "merges": int((n - 1).sum()),
                  "traffic": measured_traffic("upgma_kernel", args.workload, None),
                  "us_per_merge_step": t_tree * 1e6 / max(int(n.max()) - 1, 1),
                  "note": "one workgroup per bucket; merge steps are sequential, so the time is "
                          "the largest bucket's steps x the latency of one step"},
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def bench_psp(args):
    """Profile sum of pairs scores (Equation 4) for a batch of profile pairs:
    npairs pairs with lengths uniform in [200, 2000] columns (the range of
    the workloads' sequences), profiles of random alignments with 15% gaps,
    M = log(p_ij / (p_i p_j)) of a random symmetric joint distribution (the
    paper's PAM 200 / VTML 240 tables are not available).  One step = every
    pair's score matrix.  The kernel writes 8 bytes per score and reads
    160 bytes per column, so it is bound by HBM bandwidth."""
    import numpy as np
    import torch

    import paper_0905_1744_amd as kd

    rng = np.random.default_rng(11)
    npairs = args.pairs
    lens = rng.integers(200, 2001, size=(npairs, 2))
    x = rng.random((20, 20)) + 0.05
    P = x + x.T
    P /= P.sum()
    pm = P.sum(axis=1)
    M = np.log(P / np.outer(pm, pm))
    dev = torch.device("cuda", 0)

    def prof(L):
        return rng.dirichlet(np.ones(20), size=L) * (1 - rng.random((L, 1)) * 0.3)
    FX = torch.from_numpy(np.concatenate([prof(int(a)) for a in lens[:, 0]])).to(dev)
    FY = torch.from_numpy(np.concatenate([prof(int(b)) for b in lens[:, 1]])).to(dev)
    ctx = kd.Context(0)
    print(f"[bench] psp: {npairs} profile pairs", file=sys.stderr, flush=True)
    Md = torch.from_numpy(M).to(dev)
    S, _ = ctx.psp_scores_packed(Md, FX, lens[:, 0], FY, lens[:, 1])
    for _ in range(args.warmup):
        ctx.psp_scores_packed(Md, FX, lens[:, 0], FY, lens[:, 1], S)
    torch.cuda.synchronize()
    ctx.enable_timing(True, stages=("psp",))
    ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.psp_scores_packed(Md, FX, lens[:, 0], FY, lens[:, 1], S)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_k, n_k = ctx.stage_times()["psp"]
    ctx.enable_timing(False)
    t_k = ms_k / max(n_k, 1) / 1e3
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    scores = int((lens[:, 0] * lens[:, 1]).sum())
    nbytes = 8 * scores + 160 * int(lens.sum()) + 3200 * npairs
    gbs = nbytes / t_k / 1e9
    line = {
        "metric": "PSP column-pair scores/sec (Equation 4)", "value": scores / (ms_per_step / 1e3),
        "unit": "scores/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"psp: {npairs} profile pairs, lengths uniform [200, 2000], random "
                                f"profiles, log-odds of a random symmetric joint distribution, seed 11"),
                   "scores_per_step": scores},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                     "traffic": measured_traffic("psp", args.workload, None),
                     "kernel": "psp_g_kernel + psp_scores_kernel (one psp_scores call)", "kernel_ms": t_k * 1e3,
                     "bytes_per_launch": nbytes,
                     "flops_per_launch": 2 * 20 * scores + 2 * 400 * int(lens[:, 0].sum())},
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def batch_roofline(probes, pairs, lookups, ceiling, stages, alg_bytes, shape):
    """Roofline of the one rank launch of a batch (all sets), as for one set."""
    ms, n = stages["pairs"]
    t = ms / max(n, 1) / 1e3
    return rank_roofline(probes, pairs, lookups, t, ceiling, measured_traffic("rank_pairs_kernel", "batched", shape),
                         alg_bytes, kernel="rank_pairs_kernel (all sets in one launch)",
                         counters=profiled_counters("rank_pairs_kernel", "batched"))


def bench_batch_graph(ctx, res, off, first, Bs, args, out, t_eager):
    """The same batch as one HIP graph (kd_batch_plan): replays timed like
    the eager calls; every replay's outputs compared with the eager ones."""
    import torch
    plan = ctx.batch_plan(res, off, first, Bs, args.delta)
    for _ in range(max(args.warmup, 1)):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / args.steps
    same = all(torch.equal(plan.out[k][:out[k].numel()].view(torch.int64) if k == "ranks" else plan.out[k][:out[k].numel()],
                           out[k].view(torch.int64) if k == "ranks" else out[k]) for k in out)
    g = {"ms_per_step": t_graph * 1e3, "kernel_launches_per_replay": plan.launches,
         "identical_outputs": bool(same), "eager_ms_per_step": t_eager * 1e3,
         "launch_overhead_saved_ms": (t_eager - t_graph) * 1e3,
         "note": ("kd_batch_plan: the batch's kernels captured once into a HIP graph and replayed with "
                  "hipGraphLaunch (no host synchronization, no allocation per replay); the eager call "
                  "synchronizes once to size the layout and builds the work list on the host")}
    plan.destroy()
    print(f"[bench] batched as a graph: {t_graph * 1e3:.2f} ms per replay", file=sys.stderr, flush=True)
    return g


def bench_batched(args):
    """Many independent sets in one call (kd_batch_run) against the plain
    per-set loop (kmer_count -> kmer_rank -> sample_partition, synchronizing
    after every set) on the same device, with identical outputs required."""
    import numpy as np
    import synth
    t0 = time.perf_counter()
    sets = synth.batched(4, args.sets, workers=min(16, os.cpu_count() or 1))
    res_h, off_h, first, Bs = synth.concat(sets)
    print(f"[bench] batched workload: {len(sets)} sets, {int(first[-1])} sequences, "
          f"generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    import torch
    import paper_0905_1744_amd as kd
    dev = torch.device("cuda", 0)
    res = torch.from_numpy(res_h).to(dev)
    off = torch.from_numpy(off_h.view(np.int64)).to(dev)
    ctx = kd.Context(0)
    Ntot = int(first[-1])
    nb = int(Bs.astype(np.int64).sum()) + len(sets)
    out = dict(ranks=torch.empty(Ntot, dtype=torch.float64, device=dev),
               bucket=torch.empty(Ntot, dtype=torch.int32, device=dev),
               order=torch.empty(Ntot, dtype=torch.int32, device=dev),
               offsets=torch.empty(nb, dtype=torch.int32, device=dev))
    ns = np.diff(first.astype(np.int64))
    pairs = float((ns * (ns - 1) // 2).sum())
    tune = None
    kb = ctx.kmer_count_batch(res, off, first)
    if not args.no_autotune:  # work-list shape for batches of this size class
        best, ms = ctx.autotune(kb, args.delta)
        tune = {"tasks_per_cu": best, "ms_per_shape": ms}
    _, _, loff = kb.export_lists()
    D = np.diff(loff.cpu().numpy())
    bounds = list(zip(first[:-1].astype(np.int64), first[1:].astype(np.int64)))
    probes = sum(probe_count(D[a:b]) for a, b in bounds)
    lookups = sum(rank_lookups(D[a:b]) for a, b in bounds if b > a)
    alg_bytes = int(D.sum()) * 2 + 8 * Ntot
    ceiling = lds_ceiling(ctx)
    kb.destroy()
    for _ in range(args.warmup):
        ctx.batch_run(res, off, first, Bs, args.delta, out=out)
    torch.cuda.synchronize()
    ctx.enable_timing(True)
    ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.batch_run(res, off, first, Bs, args.delta, out=out)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    stages = ctx.stage_times()
    ctx.enable_timing(False)
    print(f"[bench] batched: {t_batch * 1e3:.2f} ms per batch", file=sys.stderr, flush=True)
    graph = bench_batch_graph(ctx, res, off, first, Bs, args, out, t_batch)
    if args.no_loop_baseline:
        line = {"metric": "batched k-mer rank + split: pair-similarities/s", "value": pairs / t_batch,
                "unit": "pair-similarities/s", "ms_per_step": t_batch * 1e3, "sets": len(sets),
                "stages_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in stages.items() if v[1]},
                "roofline": batch_roofline(probes, pairs, lookups, ceiling, stages, alg_bytes, tune["tasks_per_cu"] if tune else 32), "graph": graph}
        ctx.close()
        print(json.dumps(line), flush=True)
        return
    # per-set inputs prepared before timing (residue views, rebased offsets)
    per = []
    for q in range(len(sets)):
        a, b = int(first[q]), int(first[q + 1])
        o0, o1 = int(off_h[a]), int(off_h[b])
        per.append((res[o0:o1], (off[a:b + 1] - o0).contiguous(), b - a, int(Bs[q])))
    R1 = torch.empty(Ntot, dtype=torch.float64, device=dev)
    loop_out = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, (r, o, n, B) in enumerate(per):
        ks = ctx.kmer_count(r, o)
        Rq = ctx.kmer_rank(ks, args.delta, out=R1[int(first[q]):int(first[q]) + n])
        loop_out.append(ctx.sample_partition(Rq, B))
        ks.destroy()
        torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    print(f"[bench] per-set loop: {t_loop * 1e3:.1f} ms", file=sys.stderr, flush=True)
    same = bool(torch.equal(R1, out["ranks"]))
    ob = np.concatenate([[0], np.cumsum(Bs.astype(np.int64) + 1)])
    bb, oo, ff = out["bucket"].cpu(), out["order"].cpu(), out["offsets"].cpu()
    for q, p in enumerate(loop_out):
        a, b = int(first[q]), int(first[q + 1])
        same = same and torch.equal(p["bucket"].cpu(), bb[a:b]) and torch.equal(p["order"].cpu(), oo[a:b]) \
            and torch.equal(p["offsets"].cpu(), ff[int(ob[q]):int(ob[q + 1])])
    line = {
        "metric": "batched k-mer rank + split: pair-similarities/s and sets/s", "value": pairs / t_batch,
        "unit": "pair-similarities/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u16/f64", "data": "synthetic",
        "config": {"workload": (f"batched: {len(sets)} sets, N log-uniform [32, 2048], 4-32 families, "
                                "lognormal length mean 300, divergence 5-30%, B = min(8, N/32), seed 4"),
                   "sets": len(sets), "sequences": Ntot, "pairs": pairs, "delta": args.delta,
                   "step": "kd_batch_run (count + rank + split of every set)", "autotune": tune},
        "sets_per_s": len(sets) / t_batch,
        "per_set_loop": {"ms": t_loop * 1e3, "sets_per_s": len(sets) / t_loop, "pairs_per_s": pairs / t_loop},
        "speedup_vs_per_set_loop": t_loop / t_batch,
        "identical_outputs": same,
        "stages_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in stages.items() if v[1]},
        "roofline": batch_roofline(probes, pairs, lookups, ceiling, stages, alg_bytes, tune["tasks_per_cu"] if tune else 32),
        "graph": graph,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def plain_loop(ctx, kd, pool, pick, arr, ref, delta):
    """The plain per-job launch loop under the same arrivals: job i starts at
    max(its arrival, the previous job's end) and runs count -> rank -> split
    from host arrays with a synchronization at its end."""
    import numpy as np
    import torch
    n = len(pick)
    done = np.zeros(n)
    ok = True
    start = time.monotonic()
    for i in range(n):
        wait = start + arr[i] - time.monotonic()
        if wait > 0:
            time.sleep(wait)
        x = pool[pick[i]]
        ks = ctx.kmer_count(x.residues, x.offsets.view(np.int64))
        R = ctx.kmer_rank(ks, delta)
        p = ctx.sample_partition(R, x.B)
        got = (R.cpu().numpy(), kd.u32(p["bucket"]), kd.u32(p["order"]), kd.u32(p["offsets"]))
        ks.destroy()
        done[i] = time.monotonic() - start
        w = ref[pick[i]]
        ok = ok and all(np.array_equal(a, b) for a, b in zip(got, w))
    lat = done - arr[:n]
    return {"jobs": n, "jobs_per_s": n / done[-1], "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "identical_to_alone": bool(ok)}


def bench_served(args):
    """Poisson request streams through the server (continuous batching,
    two-stage pipeline) and through the same server limited to one job at a
    time (the FIFO loop); latency = completion - scheduled arrival.  Each
    rate offers args.jobs arrivals or args.rate_seconds of them, whichever is
    fewer (the FIFO loop at most args.fifo_seconds); arrival i carries job
    pool[k_i] of a seeded pool of distinct jobs.  Every served result is
    compared bit for bit with its job run alone through the single-set calls."""
    import numpy as np
    import synth
    rates = [float(x) for x in args.rates.split(",")]
    t0 = time.perf_counter()
    pool = synth.served_jobs(5, args.job_pool, workers=min(16, os.cpu_count() or 1))
    print(f"[bench] served workload: pool of {len(pool)} jobs, {sum(j.n for j in pool)} sequences, "
          f"generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    import paper_0905_1744_amd as kd
    ctx = kd.Context(0)
    ref = []
    for x in pool:  # each job alone through the single-set calls
        ks = ctx.kmer_count(x.residues, x.offsets.view(np.int64))
        R = ctx.kmer_rank(ks, args.delta)
        p = ctx.sample_partition(R, x.B)
        ref.append((R.cpu().numpy(), kd.u32(p["bucket"]), kd.u32(p["order"]), kd.u32(p["offsets"])))
        ks.destroy()
    pick_all = np.random.default_rng(55).integers(0, len(pool), size=args.jobs)
    results, overlap = {}, {}
    identical = True
    for mode in ("batched", "loop"):
        for lam in rates:
            cap_s = args.rate_seconds if mode == "batched" else args.fifo_seconds
            n = int(max(50, min(args.jobs, cap_s * lam)))
            pick = pick_all[:n]
            arr = synth.served_arrivals(5, n, lam)
            if mode == "loop":
                results.setdefault(mode, {})[str(int(lam) if lam.is_integer() else lam)] = \
                    plain_loop(ctx, kd, pool, pick, arr, ref, args.delta)
                r = results[mode][str(int(lam) if lam.is_integer() else lam)]
                identical = identical and r["identical_to_alone"]
                print(f"[bench] served plain loop rate {lam:g}/s, {n} jobs: p50 {r['p50_ms']:.2f} ms "
                      f"p99 {r['p99_ms']:.2f} ms, {r['jobs_per_s']:.0f} jobs/s", file=sys.stderr, flush=True)
                continue
            srv = kd.Server(0, hbm_budget=200 << 30, max_batch_seqs=args.max_batch_seqs,
                            host_arena_bytes=256 << 20, timeline=True)
            for x in pool[:2]:  # first-call costs out of the way
                srv.submit(x.residues, x.offsets, x.B, args.delta)
            got = 0
            while got < 2:
                got += len(srv.poll(8, wait_s=0.1))
            srv.timeline()
            recs, tick = {}, {}
            i = 0
            start = time.monotonic_ns()
            while len(recs) < n:
                now = time.monotonic_ns()
                while i < n and start + int(arr[i] * 1e9) <= now:
                    x = pool[pick[i]]
                    tick[srv.submit(x.residues, x.offsets, x.B, args.delta)] = i
                    i += 1
                wait = (start + int(arr[i] * 1e9) - time.monotonic_ns()) / 1e9 if i < n else 0.05
                for r in srv.poll(256, wait_s=min(max(wait, 0.0), 0.002)):
                    q = tick[r["ticket"]]
                    w = ref[pick[q]]
                    ok = r["status"] == 0 and np.array_equal(r["ranks"], w[0]) and np.array_equal(r["bucket"], w[1]) \
                        and np.array_equal(r["order"], w[2]) and np.array_equal(r["offsets"], w[3])
                    recs[q] = (r["t_done_ns"], r["batch_jobs"], ok)
            tl = srv.timeline()
            srv.close()
            lat = np.array([(recs[q][0] - start) / 1e9 - arr[q] for q in range(n)])
            end = max(v[0] for v in recs.values())
            ok = all(v[2] for v in recs.values())
            identical = identical and ok
            span = (end - start) / 1e9
            pairs = float(sum(pool[k].n * (pool[k].n - 1) / 2 for k in pick))
            key = str(int(lam) if lam.is_integer() else lam)
            results.setdefault(mode, {})[key] = {
                "jobs": n, "jobs_per_s": n / span, "pairs_per_s": pairs / span,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_batch_jobs": float(np.mean([v[1] for v in recs.values()])),
                "identical_to_alone": ok}
            if tl:
                a_ms = sum(b["count"][1] - b["count"][0] for b in tl)
                ov = 0.0
                for prev, cur in zip(tl, tl[1:]):
                    ov += max(0.0, min(cur["count"][1], prev["rank"][1]) - max(cur["count"][0], prev["rank"][0]))
                overlap[key] = {"batches": len(tl), "stage_a_ms": a_ms,
                                "stage_b_ms": sum(b["rank"][1] - b["rank"][0] for b in tl),
                                "stage_a_during_previous_stage_b_ms": ov,
                                "batches_started_during_previous_stage_b": sum(
                                    1 for prev, cur in zip(tl, tl[1:]) if cur["count"][0] < prev["rank"][1])}
            print(f"[bench] served {mode} rate {lam:g}/s, {n} jobs: p50 {results[mode][key]['p50_ms']:.2f} ms "
                  f"p99 {results[mode][key]['p99_ms']:.2f} ms, {n / span:.0f} jobs/s", file=sys.stderr, flush=True)
    top = str(int(rates[-1]) if rates[-1].is_integer() else rates[-1])
    line = {
        "metric": "served k-mer rank + split: p50/p99 request latency and jobs/s per arrival rate",
        "value": results["batched"][top]["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1,
        "steps": args.jobs, "warmup": 2, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16/f64", "data": "synthetic",
        "config": {"workload": (f"served: per rate min({args.jobs} arrivals, {args.rate_seconds:g} s of them) "
                                f"(plain per-job loop: at most {args.fifo_seconds:g} s), Poisson arrivals at "
                                f"{args.rates}/s, each a job drawn from a pool of {len(pool)}: N log-uniform "
                                "[64, 8192], 4-32 families, lognormal length mean 300, divergence 5-30%, "
                                "B = max(1, N/256), seed 5, budget 200 GiB"),
                   "delta": args.delta, "max_batch_seqs": args.max_batch_seqs},
        "rates": results, "identical_to_alone": identical,
        # throughput of the server over the plain per-job launch loop, per offered rate
        "batched_over_plain_loop": {r: results["batched"][r]["jobs_per_s"] / results["loop"][r]["jobs_per_s"]
                                    for r in results["batched"]},
        "plain_loop_note": ("each arrival, in arrival order and not before its arrival time, through "
                            "kmer_count -> kmer_rank -> sample_partition on one context from its host arrays, "
                            "results copied back, the stream synchronized before the next job"),
        "pipeline_overlap": overlap,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper20k", choices=sorted(WORKLOADS) + ["batched", "served", "global20k", "global100k",
                                                     "trees20k", "trees100k", "psp"])
    ap.add_argument("--sets", type=int, default=4096, help="batched workload: number of sets")
    ap.add_argument("--jobs", type=int, default=10000, help="served workload: arrivals per rate (at most)")
    ap.add_argument("--job-pool", type=int, default=1000, help="served workload: distinct jobs")
    ap.add_argument("--rate-seconds", type=float, default=60.0,
                    help="served workload: at most this many seconds of arrivals per rate")
    ap.add_argument("--fifo-seconds", type=float, default=20.0,
                    help="served workload: the same for the plain per-job loop")
    ap.add_argument("--max-batch-seqs", type=int, default=1 << 20,
                    help="served workload: sequences per batch")
    ap.add_argument("--pairs", type=int, default=256, help="psp workload: profile pairs")
    ap.add_argument("--rates", default="10,20,50,100,200,500,1000,2000,4000,100000",
                    help="served workload: arrival rates (jobs/s)")
    ap.add_argument("--tasks-per-cu", type=int, default=0,
                    help="rank work-list shape set by hand instead of autotuned (single-set workloads)")
    ap.add_argument("--no-loop-baseline", action="store_true",
                    help="batched workload: skip the per-set loop comparison (for profiling)")
    ap.add_argument("--delta", type=float, default=0.1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default work-list shape of the rank kernel")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times "
                         "(calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE against known bytes)")
    ap.add_argument("--lds-probe", action="store_true",
                    help="only time the random 16-bit LDS read probe (2, 8 and 32 reads in flight "
                         "per lane): the ceiling of the rank kernels' mask lookups")
    args = ap.parse_args()
    if args.lds_probe:
        import paper_0905_1744_amd as kd
        ctx = kd.Context(0)
        out = {}
        for batch in (2, 8, 32):
            ctx.calibrate_lds(1024, 4, batch)
            ms, n = ctx.calibrate_lds(1024, 64, batch)
            out[str(batch)] = {"ms": ms, "wave_reads": n, "wave_reads_per_s": n / (ms / 1e3),
                               "cu_cycles_per_wave_read_at_2.4GHz": 256 * 2.4e9 * (ms / 1e3) / n}
        ctx.close()
        print(json.dumps({"lds_probe": out, "workgroups": 1024, "reads_per_lane": 64 * 32}))
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "launches": 3}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the k-mer rank and split run on one device)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "served":
        bench_served(args)
        return
    if args.workload in ("global20k", "global100k"):
        bench_global(args)
        return
    if args.workload in ("trees20k", "trees100k"):
        bench_trees(args)
        return
    if args.workload == "psp":
        bench_psp(args)
        return

    import numpy as np
    import torch

    import paper_0905_1744_amd as kd
    import synth

    gen = {"paper20k": synth.paper20k, "small": synth.small, "large100k": synth.large100k}
    ss = gen[args.workload]()
    N, B, delta = ss.n, ss.B, args.delta
    print(f"[bench] workload {args.workload} N={N} B={B}", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    res = torch.from_numpy(ss.residues).to(dev)
    off = torch.from_numpy(ss.offsets.view(np.int64)).to(dev)
    ctx = kd.Context(0)
    R = torch.empty(N, dtype=torch.float64, device=dev)

    def step():
        kset = ctx.kmer_count(res, off)
        ctx.kmer_rank(kset, delta, out=R)
        part = ctx.sample_partition(R, B)
        return kset, part

    tune = None
    if args.tasks_per_cu:  # work-list shape set by hand (profiling a given shape)
        ctx.set_tasks_per_cu(1, N, args.tasks_per_cu)
        tune = {"tasks_per_cu": args.tasks_per_cu, "set_by_hand": True}
    for w in range(args.warmup):
        kset, _ = step()
        if w == 0 and not args.no_autotune and not args.tasks_per_cu:
            # work-list shape for this size class; later counts use it
            best, ms = ctx.autotune(kset, delta)
            tune = {"tasks_per_cu": best, "ms_per_shape": ms}
        kset.destroy()
    torch.cuda.synchronize()
    # timed region: only the rank kernel carries events (for the roofline)
    ctx.enable_timing(True, stages=("pairs",))
    ctx.reset_timing()
    kset = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if kset is not None:
            kset.destroy()
        kset, part = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pair_ms, pair_n = ctx.stage_times()["pairs"]
    # stage breakdown from a separate pass with every stage timed
    nb = min(args.steps, 5)
    ctx.enable_timing(True)
    ctx.reset_timing()
    for _ in range(nb):
        kset.destroy()
        kset, part = step()
    stages = ctx.stage_times()
    ctx.enable_timing(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    pairs = N * (N - 1) / 2
    value = pairs / (ms_per_step / 1e3)

    _, _, loff = kset.export_lists()
    D = np.diff(loff.cpu().numpy())
    probes = probe_count(D)
    t_pair = pair_ms / max(pair_n, 1) / 1e3
    achieved = probes / t_pair / 1e12
    tpc = tune["tasks_per_cu"] if tune else 32
    lookups = rank_lookups(D)
    ceiling = lds_ceiling(ctx)
    traffic = measured_traffic("rank_pairs_kernel", args.workload, tpc)
    roofline = rank_roofline(probes, pairs, lookups, t_pair, ceiling, traffic,
                             int(D.sum()) * 2 + 8 * N,
                             counters=profiled_counters("rank_pairs_kernel", args.workload))
    line = {
        "metric": METRIC, "value": value, "unit": "pair-similarities/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16/f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "N": N, "B": B, "delta": delta,
                   "step": "kmer_count + kmer_rank + sample_partition", "autotune": tune},
        "stages_ms_per_step": {k: v[0] / nb for k, v in stages.items() if v[1]},
        "stages_note": f"every stage timed with HIP events in {nb} extra steps after the timed region",
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(ss, delta, args.cpu_seconds)
        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(ss, delta, args.cpu_seconds / 2)
    kset.destroy()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
