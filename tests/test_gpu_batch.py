"""GPU parity of the batched path (pa_batch_* / pa_hash_many) against the oracle.

Every block of a batch must equal the oracle bit for bit, and the same block
hashed alone through pa_hash_async; graph replays must repeat the eager result.
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


def _device_jobs(blocks, explicit=False):
    import torch
    jobs = []
    for b in blocks:
        j = {"key": torch.from_numpy(b.key().view(np.int64)).cuda(),
             "out": torch.full((workloads.words(b.m),), -1, dtype=torch.int64, device="cuda"),
             "n": b.n, "m": b.m, "seed_a": b.seed_a, "seed_b": b.seed_b}
        if explicit:
            c = oracle.expand_operand(b.seed_a ^ 0x55, b.n, True)
            d = oracle.expand_operand(b.seed_b ^ 0x77, b.n, False)
            j["c"] = torch.from_numpy(c.view(np.int64)).cuda()
            j["d"] = torch.from_numpy(d.view(np.int64)).cuda()
            j["c_host"], j["d_host"] = c, d
        jobs.append(j)
    return jobs


def _host(t):
    return t.cpu().numpy().view(np.uint64).copy()


def _want(b, j=None):
    if j is not None and "c_host" in j:
        return oracle.pa_hash_ex(b.key(), j["c_host"], j["d_host"], b.n, b.m)
    return oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m)


def small_mixed_batch(count=48, seed=11):
    return workloads.batch_blocks(seed, count, n_lo=1, n_hi=3e5, r_lo=0.01, r_hi=1.0)


def test_mixed_batch_against_oracle(pa, ctx):
    blocks = small_mixed_batch()
    _log(f"mixed batch: n in [{min(b.n for b in blocks)}, {max(b.n for b in blocks)}]")
    jobs = _device_jobs(blocks)
    status = pa.pa_hash_many(ctx, jobs)
    assert status == [pa.PA_OK] * len(blocks)
    for b, j in zip(blocks, jobs):
        assert np.array_equal(_host(j["out"]), _want(b)), (b.n, b.m)


def test_invalid_blocks_are_skipped(pa, ctx):
    import torch
    blocks = small_mixed_batch(6, seed=5)
    jobs = _device_jobs(blocks)
    bad_m = dict(jobs[1], m=jobs[1]["n"] + 1)
    bad_n = dict(jobs[2], n=0, m=0)
    sentinel = torch.full((4,), 7, dtype=torch.int64, device="cuda")
    bad_n["out"] = sentinel
    even = _device_jobs(blocks[3:4], explicit=True)[0]
    even["c"] = torch.zeros_like(even["c"])          # c = 0 is even
    mix = [jobs[0], bad_m, bad_n, even, jobs[4], jobs[5]]
    status = pa.pa_hash_many(ctx, mix)
    assert status == [pa.PA_OK, pa.PA_EINVAL, pa.PA_EINVAL, pa.PA_EINVAL, pa.PA_OK, pa.PA_OK]
    assert _host(sentinel).tolist() == [7] * 4       # skipped block's output untouched
    for i in (0, 4, 5):
        assert np.array_equal(_host(mix[i]["out"]), _want(blocks[i]))


def test_each_block_same_alone_and_in_the_mix(pa, ctx):
    import torch
    blocks = small_mixed_batch(32, seed=12)
    jobs = _device_jobs(blocks)
    assert pa.pa_hash_many(ctx, jobs) == [pa.PA_OK] * len(blocks)
    for b, j in zip(blocks, jobs):
        alone = torch.zeros_like(j["out"])
        pa.pa_hash_async(ctx, j["key"], b.seed_a, b.seed_b, b.n, b.m, alone)
        torch.cuda.synchronize()
        assert np.array_equal(_host(alone), _host(j["out"])), (b.n, b.m)


def test_explicit_operands_in_batch(pa, ctx):
    blocks = small_mixed_batch(12, seed=13)
    jobs = _device_jobs(blocks, explicit=True)
    assert pa.pa_hash_many(ctx, jobs) == [pa.PA_OK] * len(blocks)
    for b, j in zip(blocks, jobs):
        assert np.array_equal(_host(j["out"]), _want(b, j))


def test_graph_replays_match_eager(pa, ctx):
    import torch
    blocks = small_mixed_batch(24, seed=14)
    jobs = _device_jobs(blocks)
    batch = pa.Batch(ctx, jobs)
    try:
        batch.run()
        torch.cuda.synchronize()
        eager = [_host(j["out"]) for j in jobs]
        for b, e in zip(blocks, eager):
            assert np.array_equal(e, _want(b))
        batch.capture()
        for rep in range(3):
            for j in jobs:
                j["out"].fill_(-1)                     # eager work between replays
            torch.cuda.synchronize()
            batch.run()
            torch.cuda.synchronize()
            for e, j in zip(eager, jobs):
                assert np.array_equal(_host(j["out"]), e), rep
    finally:
        batch.close()


def test_batch_workload_256_blocks(pa, ctx):
    """The batched workload itself (256 blocks, n log-uniform in [1e5, 1e7]),
    replayed through a captured graph as the benchmark does, every block
    against the oracle."""
    import torch
    blocks = workloads.batch_blocks(3, 256)
    _log(f"256-block batch: {sum(b.n for b in blocks)} bits")
    jobs = _device_jobs(blocks)
    batch = pa.Batch(ctx, jobs)
    try:
        assert batch.size() == 256
        batch.capture()
        batch.run()
        torch.cuda.synchronize()
        for i, (b, j) in enumerate(zip(blocks, jobs)):
            assert np.array_equal(_host(j["out"]), _want(b)), (i, b.n, b.m)
    finally:
        batch.close()
