"""GPU tests of the transform geometries (pa_plan_*, pa_tune).

Every geometry is a different set of kernel launches (tile sizes, rows of the
factor-3 pass, register-step splits, two or three passes); each must give the
oracle's result bit for bit.  The autotuner must keep a candidate and stay
exact, and a cached multiplier must keep the geometry it was made with.
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


def _hash(pa, ctx, torch, d_key, b):
    d_out = torch.full((workloads.words(b.m),), -1, dtype=torch.int64, device="cuda")
    pa.pa_hash_async(ctx, d_key, b.seed_a, b.seed_b, b.n, b.m, d_out)
    torch.cuda.synchronize()
    return d_out.cpu().numpy().view(np.uint64).copy()


# 2^k lengths (one and two passes) and a 3 2^k length (two and three passes,
# the radix-3 step), in both digit layouts: 40 000 and 1 000 003 bits take
# 64-bit digits (1024, 2^15); 3 200 000, 10 000 000 and 8 388 609 bits 96-bit
# digits (2^17, 2^18, 3 2^16).  The 64-bit layout's only 3 2^k length, 3 2^22,
# is covered below with closed forms.
CASES = [(40_000, 9_999), (1_000_003, 99_999), (3_200_000, 1_000_001), (10_000_000, 2_000_000),
         (8_388_609, 3_000_001)]


@pytest.mark.parametrize("n,m", CASES)
def test_every_candidate_geometry_is_exact(pa, ctx, n, m):
    import torch
    b = workloads.single_block(31, n, m)
    key = b.key()
    want = oracle.pa_hash(key, b.seed_a, b.seed_b, n, m)
    d_key = torch.from_numpy(key.view(np.int64)).cuda()
    cands = pa.pa_plan_candidates(n)
    assert cands and cands[0] == pa.pa_plan_get(ctx, n) | {"ms": 0.0}
    try:
        for c in cands:
            _log(f"plan n={n} {c}")
            pa.pa_plan_set(ctx, n, c)
            got = pa.pa_plan_get(ctx, n)
            assert (got["tile_log"], got["passes"]) == (c["tile_log"], c["passes"])
            assert np.array_equal(_hash(pa, ctx, torch, d_key, b), want), c
    finally:
        pa.pa_plan_set(ctx, n, None)


def test_five_prime_factor3_geometries_closed_form(pa, ctx):
    """n = 350 000 000 takes 64-bit digits at L = 3 2^22, the longest
    factor-3 transform: every candidate geometry against the closed form of
    the all-ones key, (c (2^n - 1) + d) mod 2^n = d - c."""
    n, m = 350_000_000, 70_000_001
    assert pa.pa_transform_length(n) == 3 << 22
    mask = (1 << n) - 1
    sa, sb = 97, 98
    c = int.from_bytes(oracle.expand_operand(sa, n, True).astype("<u8").tobytes(), "little")
    d = int.from_bytes(oracle.expand_operand(sb, n, False).astype("<u8").tobytes(), "little")
    v = ((d - c) & mask) >> (n - m)
    want = np.frombuffer(v.to_bytes(8 * workloads.words(m), "little"), dtype="<u8")
    ones = np.full(workloads.words(n), np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    cands = pa.pa_plan_candidates(n)[:12]
    assert {c_["passes"] for c_ in cands} == {2, 3}
    try:
        for cand in cands:
            _log(f"plan n={n} {cand}")
            pa.pa_plan_set(ctx, n, cand)
            got = pa.pa_hash(ctx, ones, sa, sb, n, m)
            assert np.array_equal(got, want), cand
    finally:
        pa.pa_plan_set(ctx, n, None)


def test_n1e8_geometries(pa, ctx):
    """The benchmark block under the 2-pass geometries and a few 3-pass ones."""
    import torch
    b = workloads.single("n1e8")
    d_key = torch.from_numpy(b.key().view(np.int64)).cuda()
    want = _hash(pa, ctx, torch, d_key, b)
    cands = pa.pa_plan_candidates(b.n)
    two = [c for c in cands if c["passes"] == 2]
    three = [c for c in cands if c["passes"] == 3][:4]
    try:
        for c in two + three:
            _log(f"plan n1e8 {c}")
            pa.pa_plan_set(ctx, b.n, c)
            assert np.array_equal(_hash(pa, ctx, torch, d_key, b), want), c
    finally:
        pa.pa_plan_set(ctx, b.n, None)
    _log("n1e8 oracle")
    assert np.array_equal(want, oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m))


def test_tune_keeps_a_candidate_and_stays_exact(pa, ctx):
    import torch
    b = workloads.single("n1e7")
    best = pa.pa_tune(ctx, b.n, 2)
    _log(f"tuned n1e7: {best}")
    assert best["ms"] > 0
    keys = [(c["tile_log"], c["strided_tile_log"], c["rows3_log"])
            for c in pa.pa_plan_candidates(b.n)]
    assert (best["tile_log"], best["strided_tile_log"], best["rows3_log"]) in keys
    got = pa.pa_plan_get(ctx, b.n)
    assert (got["tile_log"], got["strided_tile_log"], got["rows3_log"]) == \
        (best["tile_log"], best["strided_tile_log"], best["rows3_log"])
    d_key = torch.from_numpy(b.key().view(np.int64)).cuda()
    try:
        assert np.array_equal(_hash(pa, ctx, torch, d_key, b),
                              oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m))
    finally:
        pa.pa_plan_set(ctx, b.n, None)


def test_cached_multiplier_keeps_its_geometry(pa, ctx):
    import torch
    n, m = 3_200_000, 777_777
    b = workloads.single_block(32, n, m)
    cands = [c for c in pa.pa_plan_candidates(n) if c["passes"] == 2]
    assert len(cands) >= 2
    d_key = torch.from_numpy(b.key().view(np.int64)).cuda()
    d_out = torch.zeros(workloads.words(m), dtype=torch.int64, device="cuda")
    try:
        pa.pa_plan_set(ctx, n, cands[0])
        mul = pa.pa_mul_create(ctx, b.seed_a, n)
        pa.pa_plan_set(ctx, n, cands[-1])
        pa.pa_hash_mul_async(ctx, mul, d_key, b.seed_b, n, m, d_out)
        torch.cuda.synchronize()
        pa.pa_mul_destroy(mul)
    finally:
        pa.pa_plan_set(ctx, n, None)
    assert np.array_equal(d_out.cpu().numpy().view(np.uint64),
                          oracle.pa_hash(b.key(), b.seed_a, b.seed_b, n, m))


def test_invalid_geometry_is_rejected(pa, ctx):
    # n = 8 388 609 has a 3 * 2^16 transform: with 2^14 tiles its factor-3 pass
    # has at most 2^2 rows, so rows3_log 12 does not fit
    for n, bad in [(10**8, {"tile_log": 15}), (10**8, {"tile_log": 14, "strided_tile_log": 3}),
                   (8_388_609, {"tile_log": 14, "strided_tile_log": 14, "rows3_log": 12})]:
        with pytest.raises(pa.PAError) as e:
            pa.pa_plan_set(ctx, n, bad)
        assert e.value.status == pa.PA_EINVAL
        assert pa.pa_plan_get(ctx, n) == pa.pa_plan_candidates(n)[0]


def test_tuning_cache_file_persists_the_geometry(pa, tmp_path):
    """pa_tune appends its result to the context's tuning cache; a new context
    with the same file starts with that geometry, ignores foreign or invalid
    lines, and stays exact."""
    import torch
    path = str(tmp_path / "pa_tune.txt")
    with open(path, "w") as f:
        f.write("not a tuning line\n")
        f.write("pa_tune gfx000 2 1 15 10 10 0 1.0\n")      # another architecture
        f.write("pa_tune gfx950 2 1 15 99 10 0 1.0\n")      # invalid geometry
    n, m = 1_000_003, 99_999
    first = pa.pa_init(0, tune_cache=path)
    try:
        tuned = pa.pa_tune(first, n, 2)
    finally:
        pa.pa_destroy(first)
    lines = open(path).read().splitlines()
    assert lines[-1].startswith("pa_tune gfx950 ")
    second = pa.pa_init(0, tune_cache=path)
    try:
        got = pa.pa_plan_get(second, n)
        for k in ("tile_log", "strided_tile_log", "rows3_log"):
            assert got[k] == tuned[k], (k, got, tuned)
        b = workloads.single_block(41, n, m)
        d_key = torch.from_numpy(b.key().view(np.int64)).cuda()
        assert np.array_equal(_hash(pa, second, torch, d_key, b),
                              oracle.pa_hash(b.key(), b.seed_a, b.seed_b, n, m))
    finally:
        pa.pa_destroy(second)
    # a context without the file keeps the default geometry
    plain = pa.pa_init(0)
    try:
        assert pa.pa_plan_get(plain, n) | {"ms": 0.0} == pa.pa_plan_candidates(n)[0]
    finally:
        pa.pa_destroy(plain)


def test_hbm_budget_bounds_the_context(pa):
    """A context whose budget holds the workspace of a 10^6-bit block but not
    of a 10^8-bit one: the large block fails with PA_ENOMEM before anything is
    allocated, and the context still hashes the small block exactly."""
    import torch
    small, large = workloads.single("n1e6"), workloads.single("n1e8")
    budget = pa.pa_workspace_bytes(small.n) + (16 << 20)
    assert budget < pa.pa_workspace_bytes(large.n)
    ctx = pa.pa_init(0, hbm_budget=budget)
    try:
        held = pa.pa_ctx_bytes(ctx)
        d_large = torch.zeros(workloads.words(large.n), dtype=torch.int64, device="cuda")
        out = torch.zeros(workloads.words(large.m), dtype=torch.int64, device="cuda")
        with pytest.raises(pa.PAError) as e:
            pa.pa_hash_async(ctx, d_large, 1, 2, large.n, large.m, out)
        assert e.value.status == pa.PA_ENOMEM
        assert "budget" in pa.pa_last_error(ctx)
        assert pa.pa_ctx_bytes(ctx) == held
        d_key = torch.from_numpy(small.key().view(np.int64)).cuda()
        assert np.array_equal(_hash(pa, ctx, torch, d_key, small),
                              oracle.pa_hash(small.key(), small.seed_a, small.seed_b, small.n,
                                             small.m))
        assert pa.pa_ctx_bytes(ctx) <= budget
    finally:
        pa.pa_destroy(ctx)
    with pytest.raises(pa.PAError) as e:
        pa.pa_init(0, hbm_budget=1024)                 # cannot hold the twiddle tables
    assert e.value.status == pa.PA_ENOMEM
