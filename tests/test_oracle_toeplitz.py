"""Pins for the Toeplitz-hash oracle (oracle/toeplitz.c), all on the CPU.

The family: y = T x over GF(2) with T[i][j] = t[i - j + n - 1], t of n + m - 1
bits (the standard Toeplitz universal_2 family that the paper's Introduction
names as the common choice and its foil).  Each pin checks the oracle against
something other than its own formula: an explicit matrix, the exact collision
count of the family, unit-vector closed forms, GF(2) linearity, and an
independent floating-point FFT convolution at the n = 10^6 size.
"""
import numpy as np
import pytest

import oracle
import workloads


def bits_of(words_arr, nbits):
    w = np.asarray(words_arr, dtype=np.uint64)
    b = ((w[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.uint8)
    return b.reshape(-1)[:nbits]


def words_from_bits(b):
    b = np.asarray(b, dtype=np.uint64)
    pad = (-b.size) % 64
    b = np.concatenate([b, np.zeros(pad, dtype=np.uint64)]).reshape(-1, 64)
    return (b << np.arange(64, dtype=np.uint64)).sum(axis=1, dtype=np.uint64)


def matrix_hash(xb, tb, n, m):
    """The definition with the matrix written out: T[i][j] = t[i - j + n - 1]."""
    T = np.zeros((m, n), dtype=np.int64)
    for i in range(m):
        for j in range(n):
            T[i, j] = tb[i - j + n - 1]
    return (T @ xb.astype(np.int64)) & 1


@pytest.mark.parametrize("seed", range(6))
def test_matches_explicit_matrix(seed):
    rng = np.random.default_rng(seed)
    for _ in range(8):
        n = int(rng.integers(1, 140))
        m = int(rng.integers(1, n + 1))
        xb = rng.integers(0, 2, n).astype(np.uint8)
        tb = rng.integers(0, 2, n + m - 1).astype(np.uint8)
        got = oracle.toeplitz_ex(words_from_bits(xb), words_from_bits(tb), n, m)
        assert np.array_equal(bits_of(got, m), matrix_hash(xb, tb, n, m)), (n, m)
        # bits past m in the top output word are zero
        assert np.array_equal(got, words_from_bits(bits_of(got, m)))


@pytest.mark.parametrize("n,m", [(3, 1), (3, 3), (4, 2), (5, 3), (6, 2), (6, 4)])
def test_exact_collision_count(n, m):
    """For x != y the map t -> T(x ^ y) is GF(2)-linear and onto GF(2)^m (the
    lowest set bit j of v = x ^ y puts t[i + n - 1 - j] in row i alone among
    the still-unused bits, row by row), so exactly 2^(n+m-1-m) = 2^(n-1) of
    the 2^(n+m-1) matrices collide on every pair: the family is universal_2
    with equality."""
    for x in range(1 << n):
        for y in range(x + 1, 1 << n):
            assert oracle.toeplitz_collision_count(n, m, x, y) == 1 << (n - 1), (x, y)


def test_unit_vectors_pick_diagonals():
    """x = e_j gives y_i = t[i + n - 1 - j]; t = e_a gives y_i = x[i + n - 1 - a]."""
    rng = np.random.default_rng(7)
    n, m = 200, 77
    tb = rng.integers(0, 2, n + m - 1).astype(np.uint8)
    xb = rng.integers(0, 2, n).astype(np.uint8)
    for j in [0, 1, 63, 64, 150, n - 1]:
        e = np.zeros(n, dtype=np.uint8)
        e[j] = 1
        y = bits_of(oracle.toeplitz_ex(words_from_bits(e), words_from_bits(tb), n, m), m)
        assert np.array_equal(y, tb[np.arange(m) + n - 1 - j])
    for a in [0, 5, n - 1, n + 10, n + m - 2]:
        e = np.zeros(n + m - 1, dtype=np.uint8)
        e[a] = 1
        y = bits_of(oracle.toeplitz_ex(words_from_bits(xb), words_from_bits(e), n, m), m)
        j = np.arange(m) + n - 1 - a
        want = np.where((j >= 0) & (j < n), xb[np.clip(j, 0, n - 1)], 0)
        assert np.array_equal(y, want)


def test_linear_in_key_and_in_t():
    rng = np.random.default_rng(8)
    n, m = 1000, 333
    x1, x2 = (workloads.random_words(rng, oracle.words(n)) for _ in range(2))
    t1, t2 = (workloads.random_words(rng, oracle.words(n + m - 1)) for _ in range(2))
    h = lambda x, t: oracle.toeplitz_ex(x, t, n, m)
    assert np.array_equal(h(x1 ^ x2, t1), h(x1, t1) ^ h(x2, t1))
    assert np.array_equal(h(x1, t1 ^ t2), h(x1, t1) ^ h(x1, t2))
    assert not h(np.zeros_like(x1), t1).any()


def test_prefix_consistency_and_threads():
    """Rows i < m' use only t[0 .. n+m'-2], so a shorter output is a prefix;
    the threaded evaluation equals the single-threaded one."""
    rng = np.random.default_rng(9)
    n = 5000
    x = workloads.random_words(rng, oracle.words(n))
    full = bits_of(oracle.toeplitz(x, 1234, n, n, threads=1), n)
    for m in [1, 63, 64, 65, 1000, 4999]:
        part = bits_of(oracle.toeplitz(x, 1234, n, m, threads=5), m)
        assert np.array_equal(part, full[:m]), m


def test_sampled_bits_match_full_output():
    rng = np.random.default_rng(10)
    n, m = 3001, 1500
    x = workloads.random_words(rng, oracle.words(n))
    t = oracle.toeplitz_t(99, n, m)
    full = bits_of(oracle.toeplitz_ex(x, t, n, m), m)
    idx = rng.integers(0, m, 200)
    assert np.array_equal(oracle.toeplitz_bits(x, t, n, m, idx), full[idx])


def test_fft_convolution_at_1e6():
    """Independent evaluation at the n = 10^6 workload size: y_i is the parity of
    coefficient i + n - 1 of the integer convolution of t and x, computed with a
    float64 FFT (coefficients <= n, far inside float precision), rounded."""
    from scipy.signal import fftconvolve
    blk = workloads.single("n1e6")
    n, m = blk.n, blk.m
    x = blk.key()
    t = oracle.toeplitz_t(blk.seed_a, n, m)
    xb = bits_of(x, n).astype(np.float64)
    tb = bits_of(t, n + m - 1).astype(np.float64)
    conv = np.rint(fftconvolve(tb, xb)).astype(np.int64)
    want = conv[n - 1: n - 1 + m] & 1
    got = bits_of(oracle.toeplitz(x, blk.seed_a, n, m), m)
    assert np.array_equal(got, want)
