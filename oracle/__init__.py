"""CPU oracle for the G_{c,d} privacy-amplification hash.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the product library never imports, loads or calls it, and it
shares no code with the GPU path.

It evaluates the family of Section 2.3, eq. (6) and the g_{c,d} definition that
follows it, in the order of the pipeline of Section 3.2 (multiply-add, reduce
mod 2^n, export, keep the most significant r bits):

    V = (c*x + d) mod 2^n,   y = floor(V / 2^(n-m))

with plain limb-array arithmetic in C (``pa_oracle.c``).  Values are numpy
uint64 arrays, little-endian limb order, bit i in limb i//64 at bit i%64.

Parity pins (tests/test_oracle_pins.py): brute force at tiny n, the exact
collision count of eq. (4)/(5) for the whole family at n <= 12, algebraic
invariants with closed forms, CPython's independent big-integer arithmetic at
n up to 10^7, and published SplitMix64 known-answer values.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpa_oracle.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_splitmix64.restype = ctypes.c_uint64
    lib.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_expand_operand.restype = None
    lib.oracle_expand_operand.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_int, _u64p]
    lib.oracle_pa_hash_ex.restype = ctypes.c_int
    lib.oracle_pa_hash_ex.argtypes = [_u64p, _u64p, _u64p, ctypes.c_uint64,
                                      ctypes.c_uint64, _u64p, ctypes.c_int]
    lib.oracle_pa_hash.restype = ctypes.c_int
    lib.oracle_pa_hash.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_uint64, ctypes.c_uint64, _u64p,
                                   ctypes.c_int]
    lib.oracle_mul_full.restype = None
    lib.oracle_mul_full.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p]
    lib.oracle_mul_low.restype = None
    lib.oracle_mul_low.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p,
                                   ctypes.c_int]
    lib.oracle_collision_count.restype = ctypes.c_int64
    lib.oracle_collision_count.argtypes = [ctypes.c_uint64] * 4
    lib.oracle_toeplitz_ex.restype = ctypes.c_int
    lib.oracle_toeplitz_ex.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, _u64p,
                                       ctypes.c_int]
    lib.oracle_toeplitz.restype = ctypes.c_int
    lib.oracle_toeplitz.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    _u64p, ctypes.c_int]
    lib.oracle_toeplitz_bits.restype = ctypes.c_int
    lib.oracle_toeplitz_bits.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, _u64p,
                                         ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint8)]
    lib.oracle_toeplitz_collision_count.restype = ctypes.c_int64
    lib.oracle_toeplitz_collision_count.argtypes = [ctypes.c_uint64] * 4
    _lib = lib
    return lib


def words(bits: int) -> int:
    return (int(bits) + 63) // 64


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_u64p)


def _as_words(a, nwords: int) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    if a.ndim != 1 or a.size < nwords:
        raise ValueError(f"expected at least {nwords} uint64 words, got shape {a.shape}")
    return a


def default_par_levels(n: int) -> int:
    """Karatsuba levels to split onto threads: 2 (9 threads) for big blocks."""
    return 2 if n >= 1 << 22 else 0


def splitmix64(seed: int, i: int) -> int:
    """Output i (0-based) of SplitMix64 seeded with `seed`."""
    return int(_load().oracle_splitmix64(seed & (2**64 - 1), i))


def expand_operand(seed: int, n: int, force_odd: bool) -> np.ndarray:
    """The n-bit operand drawn from `seed` (c when force_odd, else d)."""
    out = np.zeros(words(n), dtype=np.uint64)
    _load().oracle_expand_operand(seed & (2**64 - 1), n, int(force_odd), _ptr(out))
    return out


def pa_hash_ex(key, c, d, n: int, m: int, par_levels: int | None = None) -> np.ndarray:
    """y = floor(((c x + d) mod 2^n) / 2^(n-m)) for explicit c and d."""
    w = words(n)
    key, c, d = _as_words(key, w), _as_words(c, w), _as_words(d, w)
    out = np.zeros(words(m), dtype=np.uint64)
    if par_levels is None:
        par_levels = default_par_levels(n)
    rc = _load().oracle_pa_hash_ex(_ptr(key), _ptr(c), _ptr(d), n, m, _ptr(out),
                                   par_levels)
    if rc != 0:
        raise ValueError(f"oracle rejected n={n} m={m}")
    return out


def pa_hash(key, seed_a: int, seed_b: int, n: int, m: int,
            par_levels: int | None = None) -> np.ndarray:
    """The hash with c, d expanded from seeds (c forced odd)."""
    w = words(n)
    key = _as_words(key, w)
    out = np.zeros(words(m), dtype=np.uint64)
    if par_levels is None:
        par_levels = default_par_levels(n)
    rc = _load().oracle_pa_hash(_ptr(key), seed_a & (2**64 - 1), seed_b & (2**64 - 1),
                                n, m, _ptr(out), par_levels)
    if rc != 0:
        raise ValueError(f"oracle rejected n={n} m={m}")
    return out


def mul_full(a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    assert a.size == b.size
    r = np.zeros(2 * a.size, dtype=np.uint64)
    _load().oracle_mul_full(_ptr(a), _ptr(b), a.size, _ptr(r))
    return r


def mul_low(a, b, par_levels: int = 0) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    assert a.size == b.size
    r = np.zeros(a.size, dtype=np.uint64)
    _load().oracle_mul_low(_ptr(a), _ptr(b), a.size, _ptr(r), par_levels)
    return r


def collision_count(n: int, m: int, x: int, y: int) -> int:
    """delta_G(x, y) of eq. (4) over the whole family G_{c,d} of eq. (6), n <= 20."""
    r = int(_load().oracle_collision_count(n, m, x, y))
    if r < 0:
        raise ValueError(f"bad arguments n={n} m={m}")
    return r


# ---------------------------------------------------------------------------
# Toeplitz-hash variant (toeplitz.c): y = T x over GF(2), T[i][j] = t[i - j + n - 1]
# ---------------------------------------------------------------------------

def toeplitz_t(seed_t: int, n: int, m: int) -> np.ndarray:
    """The n + m - 1 bits of t drawn from seed_t."""
    return expand_operand(seed_t, n + m - 1, False)


def _threads(threads):
    return threads if threads is not None else min(16, os.cpu_count() or 1)


def toeplitz_ex(key, t, n: int, m: int, threads: int | None = None) -> np.ndarray:
    """y = T x for explicit t of n + m - 1 bits."""
    key, t = _as_words(key, words(n)), _as_words(t, words(n + m - 1))
    out = np.zeros(words(m), dtype=np.uint64)
    if _load().oracle_toeplitz_ex(_ptr(key), _ptr(t), n, m, _ptr(out), _threads(threads)) != 0:
        raise ValueError(f"bad arguments n={n} m={m}")
    return out


def toeplitz(key, seed_t: int, n: int, m: int, threads: int | None = None) -> np.ndarray:
    """y = T x with t drawn from seed_t."""
    key = _as_words(key, words(n))
    out = np.zeros(words(m), dtype=np.uint64)
    if _load().oracle_toeplitz(_ptr(key), seed_t & (2**64 - 1), n, m, _ptr(out),
                               _threads(threads)) != 0:
        raise ValueError(f"bad arguments n={n} m={m}")
    return out


def toeplitz_bits(key, t, n: int, m: int, idx) -> np.ndarray:
    """Output bits y_i for the positions in idx (uint8 array)."""
    key, t = _as_words(key, words(n)), _as_words(t, words(n + m - 1))
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    bits = np.zeros(idx.size, dtype=np.uint8)
    rc = _load().oracle_toeplitz_bits(_ptr(key), _ptr(t), n, m, _ptr(idx), idx.size,
                                      bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise ValueError("bad arguments")
    return bits


def toeplitz_collision_count(n: int, m: int, x: int, y: int) -> int:
    """Number of the 2^(n+m-1) Toeplitz matrices with T x = T y (n + m - 1 <= 22)."""
    r = int(_load().oracle_toeplitz_collision_count(n, m, x, y))
    if r < 0:
        raise ValueError(f"bad arguments n={n} m={m}")
    return r
