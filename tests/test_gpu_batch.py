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


def test_persistent_mode_is_refused(pa, ctx):
    blocks = small_mixed_batch(4, seed=23)
    with pytest.raises(pa.PAError) as e:
        pa.Batch(ctx, _device_jobs(blocks), mode=pa.PA_BATCH_PERSISTENT)
    assert e.value.status == pa.PA_EINVAL
    assert "switched off" in pa.pa_last_error(ctx)


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


PERSISTENT_OFF = ("the persistent batch kernel hung in its first GPU runs; the cause (its queue "
                  "loop compiled so that a workgroup repeated one item) is fixed in the source "
                  "but not yet run on a GPU, so the library refuses the mode")


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_and_grouped_modes_agree(pa, ctx):
    """The persistent queue kernel and the grouped launches give the same bits
    (and the oracle's) on a mixed batch, eagerly and through graph replays."""
    import torch
    blocks = small_mixed_batch(40, seed=21)
    outs = {}
    for mode in (pa.PA_BATCH_PERSISTENT, pa.PA_BATCH_GROUPED):
        jobs = _device_jobs(blocks)
        batch = pa.Batch(ctx, jobs, mode=mode)
        try:
            assert batch.launches() == (2 if mode == pa.PA_BATCH_PERSISTENT else batch.launches())
            batch.run()
            torch.cuda.synchronize()
            assert batch.result() == pa.PA_OK
            outs[mode] = [_host(j["out"]) for j in jobs]
            batch.capture()
            for rep in range(2):
                for j in jobs:
                    j["out"].fill_(-1)
                torch.cuda.synchronize()
                batch.run()
                torch.cuda.synchronize()
                assert batch.result() == pa.PA_OK
                for e, j in zip(outs[mode], jobs):
                    assert np.array_equal(_host(j["out"]), e), (mode, rep)
        finally:
            batch.close()
    for b, p_out, g_out in zip(blocks, outs[pa.PA_BATCH_PERSISTENT], outs[pa.PA_BATCH_GROUPED]):
        assert np.array_equal(p_out, g_out), (b.n, b.m)
        assert np.array_equal(p_out, _want(b)), (b.n, b.m)


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_wait_failure_is_reported(pa, ctx):
    """Forced from the host: every dependency wait that would poll gives up at
    once.  The kernel drains (every item is taken and counted) and the run is
    reported as failed; the context and a normal batch still work after it."""
    import torch
    blocks = small_mixed_batch(16, seed=22)
    jobs = _device_jobs(blocks)
    batch = pa.Batch(ctx, jobs, force_abort=True)
    try:
        batch.run()
        torch.cuda.synchronize()
        assert batch.result() == pa.PA_EDEVICE
    finally:
        batch.close()
    jobs = _device_jobs(blocks)
    assert pa.pa_hash_many(ctx, jobs) == [pa.PA_OK] * len(blocks)
    for b, j in zip(blocks, jobs):
        assert np.array_equal(_host(j["out"]), _want(b)), (b.n, b.m)


def test_large_blocks_and_both_layouts(pa, ctx):
    """Blocks of both digit layouts (five and seven primes) and multi-pass
    transforms in one batch, against the oracle."""
    sizes = [(3_000_001, 1_000_003), (1_000_003, 99_999), (10_000_000, 2_000_000),
             (131_073, 65_537), (6_000_011, 2_999_999), (64, 64)]
    blocks = [workloads.single_block(100 + i, n, m) for i, (n, m) in enumerate(sizes)]
    jobs = _device_jobs(blocks)
    assert pa.pa_hash_many(ctx, jobs) == [pa.PA_OK] * len(blocks)
    for b, j in zip(blocks, jobs):
        assert np.array_equal(_host(j["out"]), _want(b)), (b.n, b.m)


def test_tuned_batch_stays_exact(pa, ctx):
    """pa_batch_tune picks a geometry per length group; the tuned batch, run
    eagerly and through a graph captured after tuning, equals the oracle."""
    import torch
    blocks = workloads.batch_blocks(31, 24, n_lo=1e5, n_hi=3e6)
    jobs = _device_jobs(blocks)
    batch = pa.Batch(ctx, jobs)
    try:
        before = batch.groups()
        batch.tune(2)
        after = batch.groups()
        assert [g["length"] for g in after] == [g["length"] for g in before]
        assert sum(g["blocks"] for g in after) == len(blocks)
        assert all(g["ms"] == 0.0 for g in before)
        # a group with more than one candidate geometry was timed
        assert any(g["ms"] > 0.0 for g in after)
        batch.run()
        torch.cuda.synchronize()
        for b, j in zip(blocks, jobs):
            assert np.array_equal(_host(j["out"]), _want(b)), (b.n, b.m)
        batch.capture()
        for j in jobs:
            j["out"].fill_(-1)
        torch.cuda.synchronize()
        batch.run()
        torch.cuda.synchronize()
        for b, j in zip(blocks, jobs):
            assert np.array_equal(_host(j["out"]), _want(b)), (b.n, b.m)
    finally:
        batch.close()
