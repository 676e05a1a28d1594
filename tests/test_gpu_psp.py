"""GPU: alignment profiles and the PSP score of Equation 4 (FP64 on the
matrix cores) through the C ABI against the oracle.

Bars: profiles bit-exact (count / m on both sides); scores within 1e-13 of
the oracle relative to the sum of the absolute terms (the oracle returns it
as its own PSP of |fx|, |fy|, |M|); one-hot profiles give M exactly."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

AMINO = b"ACDEFGHIKLMNPQRSTVWY"


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


def random_aln(rng, m, L, gap=0.15):
    al = np.frombuffer(AMINO + b"-.", dtype=np.uint8)
    p = np.full(22, (1 - gap) / 20)
    p[20:] = gap / 2
    return al[rng.choice(22, size=(m, L), p=p)]


def joint(rng):
    x = rng.random((20, 20)) + 0.05
    P = x + x.T
    return P / P.sum()


def check_scores(oracle_mod, M, fx, fy, S):
    want = oracle_mod.psp(fx, fy, M)
    scale = oracle_mod.psp(np.abs(fx), np.abs(fy), np.abs(M))
    err = np.abs(S - want)
    assert np.all(err <= 1e-13 * scale + 1e-300), float((err / np.maximum(scale, 1e-300)).max())


def test_profile_vs_oracle(kd, ctx, oracle_mod):
    rng = np.random.default_rng(71)
    for m, L in ((1, 1), (3, 7), (17, 255), (40, 256), (5, 1000), (300, 97)):
        say("profile", m, L)
        aln = random_aln(rng, m, L)
        f = ctx.psp_profile(aln).cpu().numpy()
        assert np.array_equal(f, oracle_mod.profile(aln))


def test_profile_errors(kd, ctx):
    aln = np.frombuffer(b"ACDE" b"AC-E" b"ACXE", dtype=np.uint8).reshape(3, 4)
    with pytest.raises(kd.KdError) as e:
        ctx.psp_profile(aln)
    assert e.value.status == -2 and (e.value.seq, e.value.pos) == (2, 2)
    with pytest.raises(kd.KdError):
        ctx.psp_profile(np.zeros((0, 4), np.uint8))


def test_psp_scores_vs_oracle(kd, ctx, oracle_mod):
    """Several pairs in one call: sizes around the 64-column tiles, single
    columns, an empty profile."""
    rng = np.random.default_rng(72)
    M = oracle_mod.psp_matrix(joint(rng))
    shapes = [(1, 1), (64, 64), (65, 63), (130, 7), (3, 200), (0, 5), (257, 129)]
    prof = [(oracle_mod.profile(random_aln(rng, 9, lx)) if lx else np.zeros((0, 20)),
             oracle_mod.profile(random_aln(rng, 13, ly)) if ly else np.zeros((0, 20))) for lx, ly in shapes]
    say("psp", shapes)
    outs = ctx.psp_scores(M, prof)
    for (fx, fy), S in zip(prof, outs):
        check_scores(oracle_mod, M, fx, fy, S.cpu().numpy())


def test_psp_one_hot_is_M(kd, ctx, oracle_mod):
    rng = np.random.default_rng(73)
    M = oracle_mod.psp_matrix(joint(rng))
    E = np.eye(20)
    S, = ctx.psp_scores(M, [(E, E)])
    assert np.array_equal(S.cpu().numpy(), M)


def test_psp_any_matrix_and_errors(kd, ctx, oracle_mod):
    """M need not be symmetric or come from a joint distribution."""
    rng = np.random.default_rng(74)
    M = rng.normal(size=(20, 20))
    fx, fy = rng.random((100, 20)), rng.random((90, 20))
    S, = ctx.psp_scores(M, [(fx, fy)])
    check_scores(oracle_mod, M, fx, fy, S.cpu().numpy())
    with pytest.raises(ValueError):
        ctx.psp_scores(np.zeros((19, 20)), [(fx, fy)])


def test_psp_packed_matches_pairs(kd, ctx, oracle_mod):
    """The packed call gives the per-pair call's scores bit for bit."""
    rng = np.random.default_rng(75)
    M = oracle_mod.psp_matrix(joint(rng))
    lx = np.array([5, 0, 300, 64, 1])
    ly = np.array([70, 9, 2, 65, 1])
    fx = [rng.random((n, 20)) for n in lx]
    fy = [rng.random((n, 20)) for n in ly]
    S, so = ctx.psp_scores_packed(M, np.concatenate(fx), lx, np.concatenate(fy), ly)
    each = ctx.psp_scores(M, list(zip(fx, fy)))
    S = S.cpu().numpy()
    for q in range(len(lx)):
        got = S[so[q]:so[q + 1]].reshape(lx[q], ly[q])
        assert np.array_equal(got, each[q].cpu().numpy())
        check_scores(oracle_mod, M, fx[q], fy[q], got)



def test_psp_scores_row_pieces_and_guards(kd, ctx, oracle_mod):
    """Row lengths around every 16- and 64-column boundary, row counts that
    leave rows past the end of a 64-row tile, outputs at offsets that put
    rows on every position within a 128-byte line: every score matches the
    oracle and no byte outside the pairs' outputs is written."""
    import torch
    rng = np.random.default_rng(76)
    M = oracle_mod.psp_matrix(joint(rng))
    ly_set = [1, 2, 15, 16, 17, 47, 48, 49, 63, 64, 65, 79, 80, 81, 127, 128, 129, 333, 2001]
    lx_set = [1, 3, 16, 17, 33, 63, 64, 65, 70]
    shapes = [(lx_set[i % len(lx_set)], ly) for i, ly in enumerate(ly_set)]
    fx = [rng.random((lx, 20)) for lx, _ in shapes]
    fy = [rng.random((ly, 20)) for _, ly in shapes]
    gap = 37  # doubles between outputs: starts drift through every line position
    total = sum(lx * ly + gap for lx, ly in shapes) + gap
    buf = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
    outs, spans, o = [], [], gap
    for lx, ly in shapes:
        outs.append(buf[o:o + lx * ly].view(lx, ly))
        spans.append((o, o + lx * ly))
        o += lx * ly + gap
    say("psp pieces", shapes)
    ctx.psp_scores(M, list(zip(fx, fy)), outs)
    host = buf.cpu().numpy()
    inside = np.zeros(total, dtype=bool)
    for (a, b), (lx, ly), x, y in zip(spans, shapes, fx, fy):
        inside[a:b] = True
        check_scores(oracle_mod, M, x, y, host[a:b].reshape(lx, ly))
    assert np.isnan(host[~inside]).all(), np.flatnonzero(~np.isnan(host) & ~inside)[:10]


def test_psp_bench_workload_sampled(kd, ctx, oracle_mod):
    """The benchmark's call at its full size: 256 profile pairs of 200 to
    2,000 columns (the same seeded recipe), one packed launch; six pairs
    checked whole, every other pair on three sampled rows."""
    import torch
    rng = np.random.default_rng(11)
    lens = rng.integers(200, 2001, size=(256, 2))
    M = oracle_mod.psp_matrix(joint(rng))

    def prof(L):
        return rng.dirichlet(np.ones(20), size=L) * (1 - rng.random((L, 1)) * 0.3)
    FX = [prof(int(a)) for a in lens[:, 0]]
    FY = [prof(int(b)) for b in lens[:, 1]]
    say("psp bench workload", int((lens[:, 0] * lens[:, 1]).sum()), "scores")
    S, so = ctx.psp_scores_packed(M, np.concatenate(FX), lens[:, 0], np.concatenate(FY), lens[:, 1])
    pick = np.random.default_rng(12)
    for q in range(256):
        lx, ly = int(lens[q, 0]), int(lens[q, 1])
        Sq = S[int(so[q]):int(so[q + 1])].view(lx, ly)
        if q % 43 == 0:
            check_scores(oracle_mod, M, FX[q], FY[q], Sq.cpu().numpy())
        else:
            rows = np.sort(pick.choice(lx, 3, replace=False))
            got = Sq[torch.from_numpy(rows).to(Sq.device)].cpu().numpy()
            check_scores(oracle_mod, M, FX[q][rows], FY[q], got)
    del S
    torch.cuda.empty_cache()
