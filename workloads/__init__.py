"""Seeded synthetic inputs for the privacy-amplification hash.

This module only draws inputs: key bits, per-job seeds, batch compositions and
arrival times.  It holds none of the hash's arithmetic, and it is the one piece
that both the GPU path's tests/benchmark and the CPU oracle's callers share.

The paper times blocks of random corrected keys of n = 10^6 .. 10^8 bits
(Section 4, Table 2) without stating their distribution; uniform random bits
stand in for them.  Every stream is SplitMix64 in counter form (Steele, Lea and
Flood, OOPSLA 2014): word i of seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15).
For a workload seed S the first three outputs of SplitMix64(S) are
(seed_key, seed_a, seed_b); the key is the stream of seed_key.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1


def splitmix64_stream(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of SplitMix64(seed) as uint64."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK64) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, i: int) -> int:
    return int(splitmix64_stream(seed, 1, i)[0])


def words(bits: int) -> int:
    return (int(bits) + 63) // 64


def key_bits(seed_key: int, n: int) -> np.ndarray:
    """An n-bit uniform key as ceil(n/64) little-endian uint64 words.

    Bits >= n of the top word are left random on purpose: the hash must ignore
    them.
    """
    return splitmix64_stream(seed_key, words(n))


def seeds_of(workload_seed: int) -> tuple[int, int, int]:
    """(seed_key, seed_a, seed_b) for a workload seed."""
    s = splitmix64_stream(workload_seed, 3)
    return int(s[0]), int(s[1]), int(s[2])


def random_words(rng: np.random.Generator, nwords: int) -> np.ndarray:
    """nwords uniform 64-bit words from a numpy generator (test inputs)."""
    return rng.integers(0, 2**64, size=nwords, dtype=np.uint64, endpoint=False)


@dataclass(frozen=True)
class Block:
    n: int
    m: int
    seed_key: int
    seed_a: int
    seed_b: int

    def key(self) -> np.ndarray:
        return key_bits(self.seed_key, self.n)


def single_block(workload_seed: int, n: int, m: int) -> Block:
    sk, sa, sb = seeds_of(workload_seed)
    return Block(n, m, sk, sa, sb)


# The three single-block workloads: (n, m, seed).  The key, the multiplier and
# the addend are uniform random bits drawn from the seed.
SINGLE_BLOCKS = {
    "n1e6": (1_000_000, 100_000, 0),
    "n1e7": (10_000_000, 2_000_000, 1),
    "n1e8": (100_000_000, 40_000_000, 2),
}


def single(name: str) -> Block:
    n, m, seed = SINGLE_BLOCKS[name]
    return single_block(seed, n, m)


def _unit(u: int) -> float:
    """Top 53 bits of a 64-bit word as a double in [0, 1)."""
    return (u >> 11) * (1.0 / (1 << 53))


def batch_blocks(workload_seed: int = 3, count: int = 256,
                 n_lo: float = 1e5, n_hi: float = 1e7,
                 r_lo: float = 0.05, r_hi: float = 0.5) -> list[Block]:
    """A batch of blocks with n log-uniform in [n_lo, n_hi] and m = round(r n),
    r uniform in [r_lo, r_hi]; every block has its own key/c/d seeds.

    Stream layout of SplitMix64(workload_seed): words 5j .. 5j+4 are
    (u_n, u_r, seed_key, seed_a, seed_b) of block j.
    """
    s = splitmix64_stream(workload_seed, 5 * count)
    out = []
    ratio = n_hi / n_lo
    for j in range(count):
        un, ur, sk, sa, sb = (int(v) for v in s[5 * j: 5 * j + 5])
        n = int(round(n_lo * ratio ** _unit(un)))
        r = r_lo + (r_hi - r_lo) * _unit(ur)
        m = max(1, min(n, int(round(r * n))))
        out.append(Block(n, m, sk, sa, sb))
    return out


def served_requests(workload_seed: int = 4, count: int = 2000,
                    n_lo: float = 1e6, n_hi: float = 1e8, ratio_m: float = 0.3,
                    rate_per_s: float = 1.0) -> tuple[list[Block], np.ndarray]:
    """Requests with n log-uniform in [n_lo, n_hi], m = round(0.3 n), and
    Poisson arrival times (exponential gaps at `rate_per_s`), in seconds.

    Stream layout: words 5j .. 5j+4 are (u_n, u_gap, seed_key, seed_a, seed_b).
    """
    s = splitmix64_stream(workload_seed, 5 * count)
    blocks, t, times = [], 0.0, []
    ratio = n_hi / n_lo
    for j in range(count):
        un, ug, sk, sa, sb = (int(v) for v in s[5 * j: 5 * j + 5])
        n = int(round(n_lo * ratio ** _unit(un)))
        m = max(1, min(n, int(round(ratio_m * n))))
        t += -math.log(1.0 - _unit(ug)) / rate_per_s
        times.append(t)
        blocks.append(Block(n, m, sk, sa, sb))
    return blocks, np.asarray(times)
