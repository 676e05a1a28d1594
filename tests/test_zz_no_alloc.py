"""sample_partition_noalloc (the split with no device allocation) against
sample_partition, through the C ABI: bit-identical outputs on consecutive
calls that reuse the library's fixed working array with shrinking inputs,
on both of the split's code paths (tiled ranking up to 8,192 samples, the
one-workgroup radix sort above), plus the oracle on the last call and the
size limit's error."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0905_1744_amd as kd
    kd.lib()
    ctx = kd.Context()
    yield kd, ctx, torch
    ctx.synchronize()
    ctx.close()


def _ranks(seed, n, tied):
    rng = np.random.default_rng(seed)
    if tied:  # few distinct values: the index breaks most comparisons
        return rng.choice(np.array([1.5, 1.75, 2.0, 2.0000000000000004]), size=n)
    return 1.9 + 0.2 * rng.random(n)


def _outs(torch, n, B, dev):
    def junk(k, dt):
        return torch.full((max(k, 1),), -1, dtype=dt, device=dev)
    return dict(bucket=junk(n, torch.int32), order=junk(n, torch.int32),
                offsets=junk(B + 1, torch.int32), pivot_rank=junk(B - 1, torch.float64),
                pivot_idx=junk(B - 1, torch.int32))


CALLS = [  # (n, B, tied): each smaller than the one before
    (300_000, 16, False),
    (20_000, 128, False),   # 16,256 samples: the radix path
    (1_000, 4, True),
]


def test_noalloc_matches_sample_partition(env):
    kd, ctx, torch = env
    import oracle
    for k, (n, B, tied) in enumerate(CALLS):
        say("sample_partition_noalloc call", k, "n", n, "B", B, "tied", tied)
        R = torch.from_numpy(_ranks(100 + k, n, tied)).to(ctx.device)
        want = ctx.sample_partition(R, B)
        got = ctx.sample_partition_noalloc(R, B, _outs(torch, n, B, ctx.device))
        ctx.synchronize()
        for key in ("bucket", "order"):
            assert torch.equal(got[key][:n], want[key]), (k, key)
        assert torch.equal(got["offsets"][:B + 1], want["offsets"]), k
        if B > 1:
            assert torch.equal(got["pivot_idx"][:B - 1], want["pivot_idx"]), k
            assert torch.equal(got["pivot_rank"][:B - 1].view(torch.int64),
                               want["pivot_rank"].view(torch.int64)), k
        if k == len(CALLS) - 1:  # same ranks on both sides: the split is exact
            p = oracle.partition(R.cpu().numpy(), B)
            assert np.array_equal(kd.u32(got["bucket"][:n]), p["bucket"])
            assert np.array_equal(kd.u32(got["order"][:n]), p["order"])
            assert np.array_equal(kd.u32(got["offsets"][:B + 1]), p["offsets"])


def test_noalloc_optional_pivots_and_size_limit(env):
    kd, ctx, torch = env
    n, B = 5_000, 8
    R = torch.from_numpy(_ranks(7, n, False)).to(ctx.device)
    want = ctx.sample_partition(R, B)
    out = _outs(torch, n, B, ctx.device)
    out["pivot_rank"] = out["pivot_idx"] = None
    say("sample_partition_noalloc without pivots n", n, "B", B)
    got = ctx.sample_partition_noalloc(R, B, out)
    ctx.synchronize()
    assert torch.equal(got["bucket"][:n], want["bucket"])
    assert torch.equal(got["order"][:n], want["order"])
    L = kd.lib()
    big = kd.lib().sample_partition_noalloc
    p = C.c_void_p(R.data_ptr())
    # checked on the host before anything is launched
    assert big(ctx.handle, p, 1048577, 4, p, p, p, None, None) == -9
    assert L.kd_strerror(-9) == b"input larger than the call's fixed maximum"
    assert big(ctx.handle, p, 100, 0, p, p, p, None, None) == -1
    assert big(ctx.handle, None, 100, 4, p, p, p, None, None) == -1
