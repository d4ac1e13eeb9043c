"""GPU parity on the method's two hardest edge cases, bit for bit.

1. Carry ripple (Alg. 1, combine and carry; Section 3.2.3, mod 2^n).  With
   d = (2^n - P) mod 2^n for P = (c x) mod 2^n every 32-bit column sum of the
   low product plus the addend is 2^32 - 1 except the lowest, which is 2^32, so
   a carry enters at bit 0 and must travel through every digit, lane, wave and
   carry chunk of the block to reach bit n, where it is discarded: V = 0.  With
   2^(n-1) added to d the same chain ends one bit short: V = 2^(n-1), so the
   output is the single top bit.  Random uniform column sums reach 2^32 - 1
   with probability about 2^-32, so seeded inputs never run these paths.
2. The CRT's largest coefficient (Section 3.2.2's product by exact
   convolution).  With x = c = 2^n - 1 every digit is at its maximum, and the
   convolution coefficient D - 1 reaches D (2^(32W) - 1)^2, the largest value
   the CRT must recover (about 1.6 bits below the seven primes' product at
   n = 301 989 888 and 2.4 bits below the five primes' at PA_MAX_N).  Since
   (2^n - 1)^2 = 1 mod 2^n, V = (1 + d) mod 2^n whatever the transform did.

Expected values are closed forms of the definition, or the oracle's (at sizes
it finishes in seconds); no expected value comes from the GPU path.  Each
case runs through pa_hash_ex (host memory) and through a batch of
explicit-operand device jobs (pa_hash_many).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

PA_MAX_N = 1 << 29


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


def _int(words):
    return int.from_bytes(np.asarray(words, dtype="<u8").tobytes(), "little")


def _words(v, n):
    w = workloads.words(n)
    return np.frombuffer((v & ((1 << (64 * w)) - 1)).to_bytes(8 * w, "little"),
                         dtype="<u8").copy()


def _top(v, n, m):
    """The output for V = v: bits n - m .. n - 1, packed from bit 0."""
    return _words((v & ((1 << n) - 1)) >> (n - m), m)


def _both_paths(pa, ctx, key, c, d, n, m):
    """(pa_hash_ex result, pa_hash_many result) for explicit operands."""
    import torch
    host = pa.pa_hash_ex(ctx, key, c, d, n, m)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()
    out = torch.full((workloads.words(m),), -1, dtype=torch.int64, device="cuda")
    job = {"key": dev(key), "c": dev(c), "d": dev(d), "out": out, "n": n, "m": m}
    torch.cuda.synchronize()
    assert pa.pa_hash_many(ctx, [job]) == [pa.PA_OK]
    got = out.cpu().numpy().view(np.uint64).copy()
    del job, out
    torch.cuda.empty_cache()
    return host, got


# 1 000 003 bits: 64-bit digits over five primes, many carry chunks;
# 3 000 001: 96-bit digits over seven primes, short chunks;
# 10^8: seven primes, 1018 long chunks (the benchmark's block);
# 301 989 888: the longest seven-prime transform (3 * 2^21);
# PA_MAX_N: the longest five-prime transform (2^24).
RIPPLE_SIZES = [1_000_003, 3_000_001, 100_000_000, 301_989_888, PA_MAX_N]


@pytest.mark.parametrize("n", RIPPLE_SIZES)
def test_carry_ripple_multiplier_one(pa, ctx, n):
    """c = 1: the low product is x itself, d = 2^n - x makes every column sum
    2^32 - 1 above the lowest, so the carry from bit 0 ripples to bit n."""
    rng = np.random.default_rng(n + 17)
    m = n // 3 + 1
    mask = (1 << n) - 1
    x = _int(workloads.random_words(rng, workloads.words(n))) & mask
    one = _words(1, n)
    d = (-x) & mask
    cases = [("x random, d = -x", x, d, 0),
             ("x random, d = 2^(n-1) - x", x, (d + (1 << (n - 1))) & mask, 1 << (n - 1)),
             ("x = 2^n - 1, d = 1", mask, 1, 0)]
    for name, xv, dv, v in cases:
        _log(f"ripple c=1 n={n}: {name}")
        want = _top(v, n, m)
        host, dev = _both_paths(pa, ctx, _words(xv, n), one, _words(dv, n), n, m)
        assert np.array_equal(host, want), name
        assert np.array_equal(dev, want), name


@pytest.mark.parametrize("n", [1_000_003, 3_000_001, 100_000_000])
def test_carry_ripple_random_product(pa, ctx, n):
    """Random odd c and random x, with d = 2^n - (c x mod 2^n) taken from the
    oracle: the ripple runs through CRT-recovered coefficients of a real
    product, and V = 0 (or 2^(n-1) with the top bit added to d)."""
    rng = np.random.default_rng(n + 29)
    m = n // 4 + 7
    mask = (1 << n) - 1
    x = workloads.random_words(rng, workloads.words(n))
    c = workloads.random_words(rng, workloads.words(n))
    c[0] |= np.uint64(1)
    zero = np.zeros(workloads.words(n), dtype=np.uint64)
    _log(f"ripple random product n={n}: oracle low product")
    p = _int(oracle.pa_hash_ex(x, c, zero, n, n)) & mask     # m = n: V itself
    d = (-p) & mask
    for name, dv, v in [("V = 0", d, 0), ("V = 2^(n-1)", (d + (1 << (n - 1))) & mask, 1 << (n - 1))]:
        _log(f"ripple random product n={n}: {name}")
        want = _top(v, n, m)
        host, dev = _both_paths(pa, ctx, x, c, _words(dv, n), n, m)
        assert np.array_equal(host, want), name
        assert np.array_equal(dev, want), name


@pytest.mark.parametrize("n", [100_000_000, 301_989_888, PA_MAX_N])
def test_crt_largest_coefficient(pa, ctx, n):
    """x = c = 2^n - 1 puts every digit at its maximum, so the middle
    convolution coefficient is the largest the primes must recover; the result
    is V = 1 + d.  d = 2^n - 1 makes that 2^n = 0 as well: the largest
    coefficients and a full-length carry in one hash."""
    rng = np.random.default_rng(n + 41)
    m = n // 5 + 3
    mask = (1 << n) - 1
    ones = _words(mask, n)
    if n in (301_989_888, PA_MAX_N):
        # both digit layouts at their longest transform, all digits full
        assert pa.pa_transform_length(n) in (3 << 21, 1 << 24)
    d = _int(workloads.random_words(rng, workloads.words(n))) & mask
    for name, dv in [("d random", d), ("d = 2^n - 1", mask)]:
        _log(f"crt max n={n}: {name}")
        want = _top(1 + dv, n, m)
        host, dev = _both_paths(pa, ctx, ones, ones, _words(dv, n), n, m)
        assert np.array_equal(host, want), name
        assert np.array_equal(dev, want), name
        if n <= 100_000_000:
            # the oracle agrees with the closed form at this size
            assert np.array_equal(oracle.pa_hash_ex(ones, ones, _words(dv, n), n, m), want)


def test_transform_lengths_of_the_edge_sizes(pa):
    assert pa.pa_transform_length(301_989_888) == 3 << 21
    assert pa.pa_transform_length(PA_MAX_N) == 1 << 24
    assert pa.pa_transform_length(100_000_000) == 1 << 21
