"""GPU parity: libpa (HIP) against the CPU oracle, bit for bit.

Every comparison is exact: the hash is an integer function of (x, c, d, n, m),
so 0 differing bits is the only passing result.  Inputs come from the shared
seeded generators; expected values come only from the oracle (or, at the
largest size, from closed forms that hold at any n).
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


def _rand_words(rng, n):
    return rng.integers(0, 2**64, workloads.words(n), dtype=np.uint64)


RAGGED = [(1, 1), (2, 1), (31, 7), (32, 32), (33, 1), (63, 63), (64, 1), (65, 64),
          (100, 99), (1000, 3), (2047, 2047), (4095, 1000), (65_536, 12_345),
          (131_071, 65_537), (131_072, 131_072), (131_073, 1), (262_145, 100_000),
          (1_000_003, 99_999), (3_000_000, 1_500_001), (4_194_305, 64),
          # sizes whose transform uses 96-bit digits over seven primes
          (3_000_001, 3), (6_000_011, 2_999_999), (8_388_609, 4_000_000)]


@pytest.mark.parametrize("n,m", RAGGED)
def test_seeded_ragged_sizes(pa, ctx, n, m):
    _log(f"seeded n={n} m={m}")
    rng = np.random.default_rng(n ^ 0x5A)
    key = _rand_words(rng, n)
    sa, sb = int(rng.integers(0, 2**63)), int(rng.integers(0, 2**63))
    got = pa.pa_hash(ctx, key, sa, sb, n, m)
    want = oracle.pa_hash(key, sa, sb, n, m)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def _int(words):
    return int.from_bytes(np.asarray(words, dtype="<u8").tobytes(), "little")


def _words(v, n):
    w = workloads.words(n)
    return np.frombuffer((v & ((1 << (64 * w)) - 1)).to_bytes(8 * w, "little"), dtype="<u8").copy()


@pytest.mark.parametrize("n,m", [(64, 64), (4097, 2000), (200_001, 77_777), (2_000_000, 1_000_000),
                                 (5_000_001, 1_000_000)])
def test_explicit_operands_and_special_keys(pa, ctx, n, m):
    _log(f"explicit n={n} m={m}")
    rng = np.random.default_rng(n)
    mask = (1 << n) - 1
    c = _rand_words(rng, n)
    c[0] |= np.uint64(1)
    d = _rand_words(rng, n)
    cases = {
        "random": _rand_words(rng, n),
        "zero": np.zeros(workloads.words(n), dtype=np.uint64),
        "one": _words(1, n),
        "all_ones": _words(mask, n),
        "power": _words(1 << (n // 3), n),
    }
    for name, key in cases.items():
        got = pa.pa_hash_ex(ctx, key, c, d, n, m)
        want = oracle.pa_hash_ex(key, c, d, n, m)
        assert np.array_equal(got, want), name
    # c = 1 and c = -1 (all ones): sums and differences, long carry/borrow chains
    key = _rand_words(rng, n)
    for cc in (_words(1, n), _words(mask, n)):
        got = pa.pa_hash_ex(ctx, key, cc, d, n, m)
        assert np.array_equal(got, oracle.pa_hash_ex(key, cc, d, n, m))


def test_argument_errors(pa, ctx):
    key = np.zeros(4, dtype=np.uint64)
    even = np.zeros(4, dtype=np.uint64)
    d = np.zeros(4, dtype=np.uint64)
    for n, m in [(0, 0), (64, 0), (64, 65)]:
        with pytest.raises(pa.PAError) as e:
            pa.pa_hash(ctx, key, 1, 2, n, m)
        assert e.value.status == pa.PA_EINVAL
    with pytest.raises(pa.PAError) as e:
        pa.pa_hash_ex(ctx, key, even, d, 200, 10)
    assert e.value.status == pa.PA_EINVAL
    with pytest.raises(pa.PAError) as e:
        pa.pa_hash(ctx, np.zeros(workloads.words(pa.PA_MAX_N + 64), dtype=np.uint64),
                   1, 2, pa.PA_MAX_N + 1, 1)
    assert e.value.status == pa.PA_EINVAL
    # the context is still usable after errors
    key = np.arange(4, dtype=np.uint64)
    assert np.array_equal(pa.pa_hash(ctx, key, 1, 2, 256, 100), oracle.pa_hash(key, 1, 2, 256, 100))


def test_workspace_reuse_shrinking_and_growing(pa, ctx):
    rng = np.random.default_rng(9)
    for n, m in [(500_000, 1000), (7_000, 6_999), (900_001, 450_000), (33, 17)]:
        _log(f"reuse n={n} m={m}")
        key = _rand_words(rng, n)
        got = pa.pa_hash(ctx, key, n, 3 * n, n, m)
        assert np.array_equal(got, oracle.pa_hash(key, n, 3 * n, n, m))


def _device_hash(pa, ctx, key_np, blk_n, blk_m, sa, sb):
    import torch
    d_key = torch.from_numpy(key_np.view(np.int64)).to("cuda")
    d_out = torch.zeros(workloads.words(blk_m), dtype=torch.int64, device="cuda")
    pa.pa_reserve(ctx, blk_n)
    pa.pa_hash_async(ctx, d_key, sa, sb, blk_n, blk_m, d_out)
    torch.cuda.synchronize()
    return d_out.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name", ["n1e6", "n1e7", "n1e8"])
def test_workload_blocks_device_path(pa, ctx, name):
    """The single-block workloads, through the device-resident entry point that
    the benchmark times, compared in full with the oracle."""
    blk = workloads.single(name)
    _log(f"workload {name} n={blk.n} m={blk.m}")
    key = blk.key()
    got = _device_hash(pa, ctx, key, blk.n, blk.m, blk.seed_a, blk.seed_b)
    want = oracle.pa_hash(key, blk.seed_a, blk.seed_b, blk.n, blk.m)
    assert np.array_equal(got, want)


def test_largest_seven_prime_transform_closed_forms(pa, ctx):
    """n = 301 989 888: 96-bit digits, D = 3 * 2^20, the longest transform of the
    seven-prime layout (3 * 2^21); closed forms that hold at any size."""
    n = 301_989_888
    assert pa.pa_transform_length(n) == 3 << 21
    m = n // 5 + 3
    mask = (1 << n) - 1
    sa, sb = 4321, 8765
    c = _int(oracle.expand_operand(sa, n, True))
    d = _int(oracle.expand_operand(sb, n, False))
    top = lambda v: _words((v & mask) >> (n - m), m)
    for name, x, v in [("one", 1, c + d), ("shift", 1 << (n - 9), (c << (n - 9)) + d),
                       ("all_ones", mask, d - c)]:
        _log(f"largest seven-prime transform key={name}")
        got = pa.pa_hash(ctx, _words(x, n), sa, sb, n, m)
        assert np.array_equal(got, top(v)), name


def test_longest_five_prime_factor3_transform_closed_forms(pa, ctx):
    """n = 350 000 000: 64-bit digits at L = 3 2^22 (96-bit digits would need
    2^23, which the seven-prime layout cannot take); closed forms."""
    n = 350_000_000
    assert pa.pa_transform_length(n) == 3 << 22
    m = n // 4 + 11
    mask = (1 << n) - 1
    sa, sb = 2468, 1357
    c = _int(oracle.expand_operand(sa, n, True))
    d = _int(oracle.expand_operand(sb, n, False))
    top = lambda v: _words((v & mask) >> (n - m), m)
    for name, x, v in [("one", 1, c + d), ("shift", 1 << (n - 5), (c << (n - 5)) + d),
                       ("all_ones", mask, d - c)]:
        _log(f"five-prime 3*2^22 key={name}")
        got = pa.pa_hash(ctx, _words(x, n), sa, sb, n, m)
        assert np.array_equal(got, top(v)), name


def test_maximum_size_closed_forms(pa, ctx):
    """n = PA_MAX_N (64-bit digits, transform length 2^24): closed forms that
    hold at any size."""
    n = pa.PA_MAX_N
    assert pa.pa_transform_length(n) == 1 << 24
    m = n // 3 + 5
    mask = (1 << n) - 1
    sa, sb = 1234, 5678
    c = _int(oracle.expand_operand(sa, n, True))
    d = _int(oracle.expand_operand(sb, n, False))
    top = lambda v: _words((v & mask) >> (n - m), m)
    for name, x, v in [("one", 1, c + d), ("shift", 1 << (n - 7), (c << (n - 7)) + d),
                       ("all_ones", mask, d - c)]:
        _log(f"max size key={name}")
        got = pa.pa_hash(ctx, _words(x, n), sa, sb, n, m)
        assert np.array_equal(got, top(v)), name
