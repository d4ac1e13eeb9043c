"""GPU tests of the Toeplitz-hash variant (pa_toeplitz, pa_toeplitz_async).

Bit-exact against the Toeplitz oracle: whole outputs at small, n = 10^6 and
n = 10^7 sizes; at n = 10^7 and n = 10^8 (two key pieces) also sampled output
bits plus properties that check every output bit (unit-vector keys select a
window of t; GF(2) linearity in the key).
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


def bit_slice(words_arr, lo, count):
    """Bits [lo, lo + count) of a word array as ceil(count/64) words."""
    w = np.asarray(words_arr, dtype=np.uint64)
    nw = (count + 63) // 64
    q, r = lo // 64, lo % 64
    src = np.concatenate([w, np.zeros(nw + 2, dtype=np.uint64)])[q: q + nw + 1]
    out = src[:nw] >> np.uint64(r)
    if r:
        out |= src[1: nw + 1] << np.uint64(64 - r)
    if count % 64:
        out[-1] &= np.uint64((1 << (count % 64)) - 1)
    return out


def test_bit_slice_helper():
    rng = np.random.default_rng(1)
    w = workloads.random_words(rng, 5)
    big = sum(int(x) << (64 * i) for i, x in enumerate(w))
    for lo, cnt in [(0, 64), (3, 100), (64, 1), (70, 250), (1, 319)]:
        want = (big >> lo) & ((1 << cnt) - 1)
        got = sum(int(x) << (64 * i) for i, x in enumerate(bit_slice(w, lo, cnt)))
        assert got == want


SMALL = [(1, 1), (2, 1), (2, 2), (63, 17), (64, 64), (65, 3), (127, 120), (1000, 999),
         (4097, 100), (20000, 12345), (131073, 5000), (1000003, 99999)]


@pytest.mark.parametrize("n,m", SMALL)
def test_small_sizes_match_oracle(pa, ctx, n, m):
    rng = np.random.default_rng(n * 7 + m)
    key = workloads.random_words(rng, oracle.words(n))
    t = workloads.random_words(rng, oracle.words(n + m - 1))
    _log(f"toeplitz explicit t n={n} m={m}")
    got = pa.pa_toeplitz(ctx, key, t, 0, n, m)
    assert np.array_equal(got[: oracle.words(m)], oracle.toeplitz_ex(key, t, n, m)), (n, m)
    seed = int(rng.integers(0, 2**63))
    got = pa.pa_toeplitz(ctx, key, None, seed, n, m)
    assert np.array_equal(got[: oracle.words(m)], oracle.toeplitz(key, seed, n, m)), (n, m)


def test_rejects_bad_sizes(pa, ctx):
    import ctypes
    key = np.zeros(4, dtype=np.uint64)
    for n, m in [(0, 1), (10, 0), (10, 11)]:
        with pytest.raises(pa.PAError) as e:
            pa.pa_toeplitz(ctx, key, None, 1, n, m)
        assert e.value.status == pa.PA_EINVAL
    # sizes past the limits are refused before any buffer is touched
    p = key.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    for n, m in [(pa.PA_MAX_N + 1, 1), (10**8, pa.PA_TOEPLITZ_MAX_M + 1)]:
        assert pa._lib.pa_toeplitz(ctx, p, None, 1, n, m, p) == pa.PA_EINVAL
    assert pa.pa_toeplitz_length(10, 11) == (0, 0)
    assert pa.pa_toeplitz_length(10**8, pa.PA_TOEPLITZ_MAX_M + 1) == (0, 0)


def test_device_entry_point_n1e6(pa, ctx):
    import torch
    blk = workloads.single("n1e6")
    key = blk.key()
    d_key = torch.from_numpy(key.view(np.int64)).cuda()
    d_out = torch.full((oracle.words(blk.m),), -1, dtype=torch.int64, device="cuda")
    _log("toeplitz async n1e6")
    pa.pa_toeplitz_async(ctx, d_key, None, blk.seed_a, blk.n, blk.m, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle.toeplitz(key, blk.seed_a, blk.n, blk.m))
    # explicit t on the device gives the same result
    t = oracle.toeplitz_t(blk.seed_a, blk.n, blk.m)
    d_t = torch.from_numpy(t.view(np.int64)).cuda()
    d_out.fill_(-1)
    pa.pa_toeplitz_async(ctx, d_key, d_t, 0, blk.n, blk.m, d_out)
    torch.cuda.synchronize()
    assert np.array_equal(d_out.cpu().numpy().view(np.uint64), got)


@pytest.mark.timeout(400)
def test_full_output_n1e7(pa, ctx):
    """The whole n = 10^7, m = 2 10^6 output against the oracle (one window
    parity per output bit, spread over every host thread)."""
    import os
    import time
    import torch
    blk = workloads.single("n1e7")
    key = blk.key()
    y = _run(pa, ctx, torch, key, blk.seed_a, blk.n, blk.m)
    threads = min(16, os.cpu_count() or 1)   # the host share of one GPU
    _log(f"toeplitz n1e7 full output: oracle on {threads} threads")
    t0 = time.perf_counter()
    want = oracle.toeplitz(key, blk.seed_a, blk.n, blk.m, threads=threads)
    _log(f"toeplitz n1e7 full output: oracle took {time.perf_counter() - t0:.1f} s")
    assert np.array_equal(y, want)


def _run(pa, ctx, torch, key, seed, n, m):
    d_key = torch.from_numpy(np.ascontiguousarray(key).view(np.int64)).cuda()
    d_out = torch.full((oracle.words(m),), -1, dtype=torch.int64, device="cuda")
    pa.pa_toeplitz_async(ctx, d_key, None, seed, n, m, d_out)
    torch.cuda.synchronize()
    return d_out.cpu().numpy().view(np.uint64).copy()


@pytest.mark.parametrize("name", ["n1e7", "n1e8"])
def test_full_size_sampled_and_properties(pa, ctx, name):
    import torch
    blk = workloads.single(name)
    n, m = blk.n, blk.m
    L, pieces = pa.pa_toeplitz_length(n, m)
    _log(f"toeplitz {name}: L={L} pieces={pieces}")
    assert L >= (n + pieces - 1) // pieces + m - 1 and L <= 3 << 25
    if name == "n1e8":
        assert pieces == 2
    key = blk.key()
    t = oracle.toeplitz_t(blk.seed_a, n, m)
    y = _run(pa, ctx, torch, key, blk.seed_a, n, m)
    # sampled output bits against the oracle, plus the first and last words
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.integers(0, m, 200), np.arange(64), np.arange(m - 64, m)])
    want = oracle.toeplitz_bits(key, t, n, m, idx)
    got = ((y[idx // 64] >> (idx % 64).astype(np.uint64)) & np.uint64(1)).astype(np.uint8)
    assert np.array_equal(got, want)
    if m % 64:
        assert int(y[-1]) >> (m % 64) == 0
    # unit keys e_j: y = bits [n - 1 - j, n - 1 - j + m) of t, every output bit
    # (j in the first and in the last key piece)
    for j in [0, 12345, n // 2 + 777, n - 1]:
        e = np.zeros(oracle.words(n), dtype=np.uint64)
        e[j // 64] = np.uint64(1) << np.uint64(j % 64)
        _log(f"toeplitz {name}: unit key j={j}")
        assert np.array_equal(_run(pa, ctx, torch, e, blk.seed_a, n, m),
                              bit_slice(t, n - 1 - j, m)), j
    # GF(2) linearity in the key, every output bit
    x2 = workloads.random_words(rng, oracle.words(n))
    y2 = _run(pa, ctx, torch, x2, blk.seed_a, n, m)
    y12 = _run(pa, ctx, torch, key ^ x2, blk.seed_a, n, m)
    assert np.array_equal(y12, y ^ y2)
