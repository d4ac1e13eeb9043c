"""Pins that tie the CPU oracle to the paper and to mathematics, not to itself.

Each check would fail for a plausible slip in the oracle: a dropped addend, a
wrong shift, a transposed operand, an even multiplier, a bad carry, a wrong
limb order or a mis-sized output.

* Known answers: a hand-worked example and published SplitMix64 outputs.
* Brute force: every (x, c, d) at n <= 5 and every m, with Python integers.
* Universality, eq. (3)-(5): for the whole family G_{c,d} of eq. (6) the
  collision count of every pair x != y has the closed form derived below, which
  meets the bound |G|/|B| of eq. (5) with equality.
* Closed-form special cases and algebraic invariants (key 0 / 1 / all-ones /
  2^k, c = 1 / -1, affine in d, additive in x, commutative, slice consistency).
* CPython's independent big-integer multiply at sizes up to n = 10^7.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def to_int(words) -> int:
    return int.from_bytes(np.asarray(words, dtype="<u8").tobytes(), "little")


def to_words(v: int, nbits: int) -> np.ndarray:
    w = oracle.words(nbits)
    return np.frombuffer(v.to_bytes(8 * w, "little"), dtype="<u8").copy()


def hx(x: int, c: int, d: int, n: int, m: int) -> int:
    return to_int(oracle.pa_hash_ex(to_words(x, n), to_words(c, n), to_words(d, n), n, m))


def rand_int(rng, bits: int) -> int:
    return to_int(rng.integers(0, 2**64, oracle.words(bits), dtype=np.uint64)) & ((1 << bits) - 1)


# --------------------------------------------------------------------------
# known answers
# --------------------------------------------------------------------------

def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield [int(t) for t in line.split()]


def test_splitmix64_known_answers():
    rows = list(_rows("splitmix64_kat.txt"))
    assert len(rows) == 5
    for seed, i, want in rows:
        assert oracle.splitmix64(seed, i) == want
        # the shared input generator implements the same published definition
        assert workloads.splitmix64(seed, i) == want


def test_hand_worked_examples():
    rows = list(_rows("hand_example.txt"))
    assert len(rows) == 4
    for n, m, x, c, d, y in rows:
        assert hx(x, c, d, n, m) == y


def test_expand_operand_layout():
    # c is the SplitMix64 stream of seed_a, masked to n bits, bit 0 set
    n = 130
    c = oracle.expand_operand(99, n, True)
    d = oracle.expand_operand(99, n, False)
    raw = [oracle.splitmix64(99, i) for i in range(3)]
    assert int(d[0]) == raw[0] and int(d[1]) == raw[1] and int(d[2]) == raw[2] & 3
    assert int(c[0]) == raw[0] | 1 and int(c[2]) == raw[2] & 3


# --------------------------------------------------------------------------
# brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_tiny(n):
    mask = (1 << n) - 1
    for m in range(1, n + 1):
        for x in range(1 << n):
            for c in range(1 << n):
                for d in range(1 << n):
                    want = ((c * x + d) & mask) >> (n - m)
                    assert hx(x, c, d, n, m) == want, (n, m, x, c, d)


def test_random_small_sizes_against_python_int():
    rng = np.random.default_rng(1)
    for _ in range(300):
        n = int(rng.integers(1, 600))
        m = int(rng.integers(1, n + 1))
        x, c, d = rand_int(rng, n), rand_int(rng, n) | 1, rand_int(rng, n)
        assert hx(x, c, d, n, m) == ((c * x + d) & ((1 << n) - 1)) >> (n - m)


def test_input_bits_above_n_are_ignored():
    rng = np.random.default_rng(2)
    n, m = 1000, 300
    key = rng.integers(0, 2**64, oracle.words(n), dtype=np.uint64)
    c = rng.integers(0, 2**64, oracle.words(n), dtype=np.uint64) | np.uint64(1)
    d = rng.integers(0, 2**64, oracle.words(n), dtype=np.uint64)
    y1 = oracle.pa_hash_ex(key, c, d, n, m)
    mask = to_words((1 << n) - 1, n)
    y2 = oracle.pa_hash_ex(key & mask, c & mask, d & mask, n, m)
    assert np.array_equal(y1, y2)
    assert to_int(y1) < (1 << m)


# --------------------------------------------------------------------------
# universality: exact collision counts, eq. (3)-(5)
# --------------------------------------------------------------------------

def nu2(v: int) -> int:
    return (v & -v).bit_length() - 1


def closed_form_collisions(n: int, m: int, x: int, y: int) -> int:
    """#{(c odd, d) in Z_{2^n}^2 : g(x) = g(y)} for x != y.

    With s = n - m and delta = c (x - y) mod 2^n, the number of d that keep x
    and y in the same output bucket is 2^m max(0, 2^s - dist(delta)), dist the
    distance to 0 on the cycle Z_{2^n}.  For t = nu2(x - y) < s, as c runs over
    the odd residues delta runs over 2^t * (odd o < 2^(n-t)), each 2^t times,
    and the sum over o is 2^(2s-t-1); so the total is 2^(2n-1-m).  For t >= s
    every delta is at distance >= 2^s and the count is 0.
    """
    t = nu2((x - y) % (1 << n))
    return (1 << (2 * n - 1 - m)) if t < n - m else 0


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (3, 1), (3, 2), (4, 1), (4, 2), (4, 3),
                                 (5, 2), (5, 4), (6, 1), (6, 3), (6, 5)])
def test_collision_count_all_pairs(n, m):
    family = (1 << (n - 1)) * (1 << n)          # |G|: c odd, d any
    bound = family // (1 << m)                 # |G| / |B|, eq. (5)
    for x in range(1 << n):
        for y in range(x + 1, 1 << n):
            got = oracle.collision_count(n, m, x, y)
            assert got == closed_form_collisions(n, m, x, y), (x, y, got)
            assert got <= bound


@pytest.mark.parametrize("n,m", [(10, 3), (12, 5)])
def test_collision_count_sampled_pairs(n, m):
    rng = np.random.default_rng(n)
    pairs = [(0, 1), (0, 1 << (n - m - 1)), (0, 1 << (n - m)), (3, (1 << n) - 1)]
    for _ in range(2):
        x, y = (int(v) for v in rng.integers(0, 1 << n, 2))
        if x != y:
            pairs.append((x, y))
    for x, y in pairs:
        assert oracle.collision_count(n, m, x, y) == closed_form_collisions(n, m, x, y)


def test_even_multiplier_breaks_universality():
    # eq. (6) requires gcd(c, 2) = 1.  With c even, x = 0 and x = 2^(n-1)
    # collide for every (c, d): check it on the oracle's own evaluation.
    n, m = 6, 3
    for c in range(0, 1 << n, 2):
        for d in range(1 << n):
            assert hx(0, c, d, n, m) == hx(1 << (n - 1), c, d, n, m)


# --------------------------------------------------------------------------
# closed forms and invariants at ragged sizes
# --------------------------------------------------------------------------

SIZES = [(64, 64), (65, 1), (1000, 999), (4127, 1000), (33 * 64 + 5, 17),
         (100_003, 31_999), (262_144, 65_536)]


@pytest.mark.parametrize("n,m", SIZES)
def test_special_keys(n, m):
    rng = np.random.default_rng(n)
    mask = (1 << n) - 1
    c, d = rand_int(rng, n) | 1, rand_int(rng, n)
    top = lambda v: (v & mask) >> (n - m)
    assert hx(0, c, d, n, m) == top(d)                     # key 0: the addend
    assert hx(1, c, d, n, m) == top(c + d)                 # key 1: c + d
    assert hx(mask, c, d, n, m) == top(d - c)              # all ones = -1
    k = int(rng.integers(0, n))
    assert hx(1 << k, c, d, n, m) == top((c << k) + d)     # shifted product
    x = rand_int(rng, n)
    assert hx(x, 1, d, n, m) == top(x + d)                 # c = 1
    assert hx(x, mask, d, n, m) == top(d - x)              # c = -1


@pytest.mark.parametrize("n,m", SIZES)
def test_invariants(n, m):
    rng = np.random.default_rng(n + 1)
    mask = (1 << n) - 1
    x1, x2, d = rand_int(rng, n), rand_int(rng, n), rand_int(rng, n)
    c = rand_int(rng, n) | 1
    v = lambda x, cc, dd: hx(x, cc, dd, n, n)
    # affine in d
    assert v(x1, c, d) == (v(x1, c, 0) + d) & mask
    # additive in x
    assert v((x1 + x2) & mask, c, 0) == (v(x1, c, 0) + v(x2, c, 0)) & mask
    # operand symmetry
    xo = x1 | 1
    assert v(xo, c, d) == v(c, xo, d)
    # the m-bit output is the top of the full n-bit value
    assert hx(x1, c, d, n, m) == v(x1, c, d) >> (n - m)


# --------------------------------------------------------------------------
# independent big-integer arithmetic (CPython) at the workload sizes
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["n1e6", "n1e7"])
def test_workload_blocks_against_python_int(name):
    blk = workloads.single(name)
    key = blk.key()
    y = oracle.pa_hash(key, blk.seed_a, blk.seed_b, blk.n, blk.m)
    mask = (1 << blk.n) - 1
    x = to_int(key) & mask
    c = to_int(oracle.expand_operand(blk.seed_a, blk.n, True))
    d = to_int(oracle.expand_operand(blk.seed_b, blk.n, False))
    assert c & 1 == 1
    assert to_int(y) == ((c * x + d) & mask) >> (blk.n - blk.m)


def test_low_product_against_python_int():
    rng = np.random.default_rng(5)
    for w in [1, 31, 32, 33, 63, 64, 65, 127, 1000, 4095, 4096, 4097, 20_000]:
        a = rng.integers(0, 2**64, w, dtype=np.uint64)
        b = rng.integers(0, 2**64, w, dtype=np.uint64)
        a[-1] = np.uint64(2**64 - 1)
        full = to_int(a) * to_int(b)
        assert to_int(oracle.mul_full(a, b)) == full
        assert to_int(oracle.mul_low(a, b)) == full & ((1 << (64 * w)) - 1)
        if w >= 4096:
            assert to_int(oracle.mul_low(a, b, par_levels=2)) == full & ((1 << (64 * w)) - 1)
