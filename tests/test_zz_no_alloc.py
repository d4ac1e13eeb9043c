"""The allocation-free entry point (pa_hash_async_noalloc) against pa_hash_async.

Two calls in a row through the C ABI, the second on a smaller block, each
compared bit for bit with pa_hash_async on the same inputs (and the small one
with the oracle); the device's free memory is the same before and after the
calls, and a block too large for the fixed scratch is refused.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pa():
    import paper_1910_04429_amd as pa
    return pa


@pytest.fixture(scope="module")
def ctx(pa):
    c = pa.pa_init(0)
    yield c
    pa.pa_destroy(c)


def _host(t):
    return t.cpu().numpy().view(np.uint64).copy()


def test_noalloc_matches_hash_async_on_two_calls(pa, ctx):
    import torch
    blocks = [workloads.single("n1e8"), workloads.single_block(7, 1_000_003, 250_001)]
    dev = [(torch.from_numpy(b.key().view(np.int64)).cuda(),
            torch.full((workloads.words(b.m),), -1, dtype=torch.int64, device="cuda"),
            torch.full((workloads.words(b.m),), -1, dtype=torch.int64, device="cuda"))
           for b in blocks]
    # the reference results first: this also grows the context's workspace
    # and lets the runtime set up its launch resources before the free
    # memory is read
    for b, (key, _, ref) in zip(blocks, dev):
        _log(f"pa_hash_async n={b.n} m={b.m}")
        pa.pa_hash_async(ctx, key, b.seed_a, b.seed_b, b.n, b.m, ref)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for b, (key, out, _) in zip(blocks, dev):
        _log(f"noalloc n={b.n} m={b.m}")
        pa.pa_hash_async_noalloc(ctx, key, b.seed_a, b.seed_b, b.n, b.m, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0      # nothing was allocated
    for b, (key, out, ref) in zip(blocks, dev):
        assert np.array_equal(_host(out), _host(ref)), b.n
    small = blocks[1]
    assert np.array_equal(_host(dev[1][1]),
                          oracle.pa_hash(small.key(), small.seed_a, small.seed_b, small.n, small.m))


def test_noalloc_refuses_blocks_beyond_the_scratch(pa, ctx):
    import torch
    n, m = 150_000_000, 1000
    assert pa.pa_workspace_bytes(n) > pa.PA_NOALLOC_MAX_BYTES
    key = torch.zeros(workloads.words(n), dtype=torch.int64, device="cuda")
    out = torch.full((workloads.words(m),), 5, dtype=torch.int64, device="cuda")
    with pytest.raises(pa.PAError) as e:
        pa.pa_hash_async_noalloc(ctx, key, 1, 2, n, m, out)
    assert e.value.status == pa.PA_EINVAL
    assert "PA_NOALLOC_MAX_BYTES" in pa.pa_last_error(ctx)
    torch.cuda.synchronize()
    assert _host(out).tolist() == [5] * workloads.words(m)
