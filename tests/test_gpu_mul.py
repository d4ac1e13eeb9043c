"""GPU parity of the cached-multiplier path (pa_mul_*): one transform of c,
many keys; every result must equal the oracle with that c."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pa():
    import paper_1910_04429_amd as pa
    return pa


@pytest.fixture(scope="module")
def ctx(pa):
    c = pa.pa_init(0)
    yield c
    pa.pa_destroy(c)


@pytest.mark.parametrize("n,m", [(1000, 999), (131_073, 20_000), (1_000_000, 100_000),
                                 (10_000_000, 2_000_000)])
def test_seeded_multiplier_many_keys(pa, ctx, n, m):
    import torch
    rng = np.random.default_rng(n)
    seed_a = int(rng.integers(0, 2**63))
    mul = pa.pa_mul_create(ctx, seed_a, n)
    try:
        for r in range(3):
            key = rng.integers(0, 2**64, workloads.words(n), dtype=np.uint64)
            seed_b = int(rng.integers(0, 2**63))
            d_key = torch.from_numpy(key.view(np.int64)).cuda()
            d_out = torch.zeros(workloads.words(m), dtype=torch.int64, device="cuda")
            pa.pa_hash_mul_async(ctx, mul, d_key, seed_b, n, m, d_out)
            torch.cuda.synchronize()
            got = d_out.cpu().numpy().view(np.uint64)
            assert np.array_equal(got, oracle.pa_hash(key, seed_a, seed_b, n, m)), r
    finally:
        pa.pa_mul_destroy(mul)


def test_explicit_multiplier(pa, ctx):
    import torch
    n, m = 70_001, 35_000
    rng = np.random.default_rng(3)
    c = oracle.expand_operand(99, n, True)
    d_c = torch.from_numpy(c.view(np.int64)).cuda()
    mul = pa.pa_mul_create(ctx, 0, n, c=d_c)
    try:
        key = rng.integers(0, 2**64, workloads.words(n), dtype=np.uint64)
        d_key = torch.from_numpy(key.view(np.int64)).cuda()
        d_out = torch.zeros(workloads.words(m), dtype=torch.int64, device="cuda")
        pa.pa_hash_mul_async(ctx, mul, d_key, 5, n, m, d_out)
        torch.cuda.synchronize()
        d = oracle.expand_operand(5, n, False)
        assert np.array_equal(d_out.cpu().numpy().view(np.uint64),
                              oracle.pa_hash_ex(key, c, d, n, m))
    finally:
        pa.pa_mul_destroy(mul)
    even = torch.zeros(workloads.words(n), dtype=torch.int64, device="cuda")
    with pytest.raises(pa.PAError) as e:
        pa.pa_mul_create(ctx, 0, n, c=even)
    assert e.value.status == pa.PA_EINVAL


def test_multiplier_outlives_its_context_and_serves_another(pa):
    """A multiplier made on one context hashes through a second context on
    the same device, and is freed after its creating context is gone."""
    import torch
    n, m = 200_003, 60_000
    rng = np.random.default_rng(8)
    key = rng.integers(0, 2**64, workloads.words(n), dtype=np.uint64)
    d_key = torch.from_numpy(key.view(np.int64)).cuda()
    d_out = torch.zeros(workloads.words(m), dtype=torch.int64, device="cuda")
    first = pa.pa_init(0)
    mul = pa.pa_mul_create(first, 41, n)
    torch.cuda.synchronize()
    pa.pa_destroy(first)
    second = pa.pa_init(0)
    try:
        pa.pa_hash_mul_async(second, mul, d_key, 42, n, m, d_out)
        torch.cuda.synchronize()
    finally:
        pa.pa_mul_destroy(mul)
        pa.pa_destroy(second)
    assert np.array_equal(d_out.cpu().numpy().view(np.uint64), oracle.pa_hash(key, 41, 42, n, m))
