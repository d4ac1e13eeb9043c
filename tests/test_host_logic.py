"""Host-side logic that needs no GPU: the server's HBM arena (admission by
footprint) and the transform plan exported by the library."""
import os
import subprocess

import numpy as np
import pytest
import torch  # noqa: F401  (load torch's HIP runtime before libpa, as the binding does)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_04429_amd", "csrc")

DRIVER = r"""
#include <stdio.h>
#include "arena.h"
int main() {
    unsigned long long size; if (scanf("%llu", &size) != 1) return 2;
    pa::Arena a(size);
    char op; unsigned long long x, y;
    while (scanf(" %c", &op) == 1) {
        if (op == 'a') { if (scanf("%llu", &x) != 1) return 2; uint64_t off = 0;
            if (a.alloc(x, &off)) printf("ok %llu\n", (unsigned long long)off); else printf("full\n"); }
        else if (op == 'f') { if (scanf("%llu %llu", &x, &y) != 2) return 2; a.release(x, y); printf("freed\n"); }
        else if (op == 'p') { printf("peak %llu\n", (unsigned long long)a.peak()); }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def arena_bin(tmp_path_factory):
    d = tmp_path_factory.mktemp("arena")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def run(exe, size, ops):
    text = f"{size}\n" + "\n".join(ops) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return out.split("\n")[:-1]


def r256(x):
    return (x + 255) // 256 * 256


def test_arena_random_alloc_free_never_overlaps(arena_bin):
    """Random allocations and frees: every block is 256-aligned, in range and
    disjoint from every live block; the reported peak matches a model."""
    rng = np.random.default_rng(0)
    size = 1 << 24
    ops, live, used, peak = [], [], 0, 0
    for _ in range(150):
        if live and rng.random() < 0.45:
            off, sz = live.pop(int(rng.integers(len(live))))
            ops.append(f"f {off} {sz}")
            used -= sz
            continue
        want = int(rng.integers(1, 1 << 21))
        ops.append(f"a {want}")
        res = run(arena_bin, size, ops)[-1]
        if not res.startswith("ok"):
            ops.pop()                      # a refused request changes nothing
            continue
        off, sz = int(res.split()[1]), r256(want)
        assert off % 256 == 0 and off + sz <= size
        for o2, s2 in live:
            assert off + sz <= o2 or o2 + s2 <= off, "overlapping blocks"
        live.append((off, sz))
        used += sz
        peak = max(peak, used)
    assert run(arena_bin, size, ops + ["p"])[-1] == f"peak {peak}"


def test_arena_coalesces_back_to_one_block(arena_bin):
    size = 1 << 20
    ops = [f"a {4096}" for _ in range(256)]          # fill exactly
    ops.append("a 1")                                 # no room
    offs = list(range(0, size, 4096))
    rng = np.random.default_rng(1)
    for o in rng.permutation(offs):
        ops.append(f"f {o} 4096")
    ops.append(f"a {size}")                           # whole range again
    out = run(arena_bin, size, ops)
    assert out[255].startswith("ok") and out[256] == "full"
    assert out[-1] == "ok 0"


def test_arena_first_fit_and_merge(arena_bin):
    size = 10 * 256
    out = run(arena_bin, size, ["a 512", "a 512", "a 512", "f 512 512", "a 1024",
                                "f 0 512", "a 1024"])
    # after freeing [512, 1024) the free pieces [512, 1024) and [1536, 2560) are
    # apart; a 1024-byte request takes the first piece that fits ...
    assert out[0] == "ok 0" and out[1] == "ok 512" and out[2] == "ok 1024"
    assert out[4] == "ok 1536"
    # ... and freeing [0, 512) merges with [512, 1024) into a 1024-byte piece
    assert out[6] == "ok 0"


def _shortest_length(need):
    """Smallest 2^k (k >= 6) >= need, or, from 2^18 on, 3 * 2^(k-2) when that fits."""
    k = max(6, (need - 1).bit_length())
    if k >= 18 and 3 << (k - 2) >= need:
        return 3 << (k - 2)
    return 1 << k


def test_plan_lengths_cover_the_linear_convolution():
    """The layout with less transform work (primes x L x log2 L) among 64-bit
    digits over five primes and 96-bit digits over seven (only lengths that
    divide 3 * 2^22, the order of the last two primes' roots), each with the
    shortest L >= 2D - 1 of the form 2^k or 3 * 2^k."""
    import math
    import paper_1910_04429_amd as pa
    order = 3 << 25
    seen = set()
    for n in [1, 63, 64, 65, 1000, 65_536, 1_000_000, 5_000_000, 6_291_400, 6_400_000, 10**7,
              3 * 10**7, 10**8, 2 * 10**8, 301_989_888, 301_989_889, 350_000_000, 402_653_184,
              pa.PA_MAX_N] + \
            [int(x) for x in np.geomspace(1e5, pa.PA_MAX_N, 40)]:
        cands = []
        for W, P, root_order in [(2, 5, order), (3, 7, 3 << 22)]:
            D = (n + 32 * W - 1) // (32 * W)
            L = _shortest_length(2 * D - 1)
            assert L >= 2 * D - 1 and order % L == 0
            if root_order % L == 0:
                cands.append((P * L * math.log2(L), W, P, L))
        work, W, P, L = min(cands, key=lambda c: (c[0], c[1]))
        assert pa.pa_transform_length(n) == L, n
        assert pa.pa_workspace_bytes(n) >= 2 * P * 4 * L
        seen.add(W)
    assert seen == {2, 3}
    assert pa.pa_transform_length(10**6) == 1 << 15        # 64-bit digits, five primes
    assert pa.pa_transform_length(10**8) == 1 << 21        # 96-bit digits, seven primes
    # the largest seven-prime transform; 2^23 (n up to 402 653 184 with 96-bit
    # digits) does not divide 3 * 2^22, so those blocks take 64-bit digits
    assert pa.pa_transform_length(301_989_888) == 3 << 21
    assert pa.pa_transform_length(350_000_000) == 3 << 22


def test_carry_sums_fit_in_the_multiplier_spectrum():
    """The carry kernels keep the output window's column sums in the
    multiplier spectrum's array (free after the pointwise product): a low word
    per 32-bit digit (D of them, padded to 64), then a word of high bits per
    carry thread (4 or more digits each).  That array holds (2 W + 1) L >= 5 L
    words for every block size, the smallest transforms included."""
    import paper_1910_04429_amd as pa
    for n in list(range(1, 4200, 37)) + [65_536, 1_000_003, 10**8, 301_989_888, 350_000_000,
                                          pa.PA_MAX_N] + \
            [int(x) for x in np.geomspace(1e4, pa.PA_MAX_N, 60)]:
        D = (n + 31) // 32
        need = ((D + 63) // 64) * 64 + (D + 3) // 4
        assert need <= 5 * pa.pa_transform_length(n), n


def _write_counter_csv(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as f:
        f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for disp, name, val in rows:
            f.write(f'{disp},"{name}","{counter}",{val}\n')


def test_counter_ingest_scales_by_the_calibration_kernel(tmp_path):
    """bench.py's counter ingest: per-launch k_pass bytes = mean FETCH (KiB) x
    (known calibration KiB / calibration FETCH) + the same for WRITE, over the
    k_pass launches of the last three hashes (runs ended by a carry kernel)."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    calib = "at::native::bitwise_not_kernel"
    kp, kc = "pa::k_pass(pa::PassArgs)", "pa::k_carry<8, true>(pa::CarryArgs)"

    def seq(values_per_pass):
        rows, d = [(1, calib, None)], 2
        for _ in range(4):                               # four hashes of four passes
            for v in values_per_pass:
                rows.append((d, kp, v)); d += 1
            rows.append((d, kc, 1.0)); d += 1
        return rows
    fetch = [(i, n, 1024.0 if v is None else v) for i, n, v in seq([100.0, 200.0, 300.0, 400.0])]
    write = [(i, n, 4096.0 if v is None else v) for i, n, v in seq([50.0] * 4)]
    _write_counter_csv(tmp_path / "f", "FETCH_SIZE", fetch)
    _write_counter_csv(tmp_path / "w", "WRITE_SIZE", write)
    _write_counter_csv(tmp_path / "s", "SQ_INSTS_VALU",
                       [(i, n, 7.0 if v is None else v) for i, n, v in seq([10.0, 30.0, 10.0, 30.0])])
    out = bench.ingest_counters([str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "s")],
                                4, path=str(tmp_path / "c.json"))
    # 4 MiB = 4096 KiB known: fetch factor 4, write factor 1
    assert out["calibration"]["fetch_factor"] == 4.0 and out["calibration"]["write_factor"] == 1.0
    assert out["passes_per_hash"] == 4
    assert out["fetch_kib_per_pass"] == [100.0, 200.0, 300.0, 400.0]
    assert out["bytes_per_launch"] == int(250.0 * 1024 * 4 + 50.0 * 1024)
    assert out["sq"]["SQ_INSTS_VALU"] == 20.0
    assert out["sq_per_pass"]["SQ_INSTS_VALU"] == [10.0, 30.0, 10.0, 30.0]


def test_toeplitz_plan_covers_the_needed_slice():
    """Each key piece of width w needs cyclic length L >= w + m - 1 (positions
    w - 1 .. w + m - 2 of the convolution are then free of wrap-around); L is
    2^k or 3 * 2^k and at most 3 * 2^25; the pieces cover the key."""
    import paper_1910_04429_amd as pa
    for n, m in [(1, 1), (64, 1), (1000, 1000), (10**6, 10**5), (10**7, 2 * 10**6),
                 (10**8, 4 * 10**7), (60_000_000, 50_000_000), (pa.PA_MAX_N, 1),
                 (pa.PA_MAX_N, pa.PA_TOEPLITZ_MAX_M)]:
        L, pieces = pa.pa_toeplitz_length(n, m)
        width = -(-n // pieces)
        assert pieces >= 1 and pieces * width >= n and (pieces - 1) * width < n
        assert width + m - 1 <= L <= 3 << 25
        f = 3 if L % 3 == 0 else 1
        assert (L // f) & (L // f - 1) == 0
    assert pa.pa_toeplitz_length(10**8, 4 * 10**7) == (3 << 25, 2)
    assert pa.pa_toeplitz_length(10**6, 10**5) == (3 << 19, 1)
    assert pa.pa_toeplitz_length(5, 6) == (0, 0)


def test_plan_candidates_default_first_and_valid():
    import paper_1910_04429_amd as pa
    c8 = pa.pa_plan_candidates(10**8)
    assert (c8[0]["tile_log"], c8[0]["strided_tile_log"], c8[0]["rows3_log"], c8[0]["passes"]) \
        == (12, 12, 0, 2)
    keys = {(c["tile_log"], c["strided_tile_log"], c["rows3_log"]) for c in c8}
    assert (13, 13, 0) in keys and (14, 14, 0) in keys and len(keys) == len(c8)
    assert all(2 <= c["passes"] <= 3 for c in c8)
    small = pa.pa_plan_candidates(1000)
    assert small and all(c["passes"] == 1 for c in small)
    assert pa.pa_plan_candidates(0) == [] and pa.pa_plan_candidates(pa.PA_MAX_N + 1) == []
