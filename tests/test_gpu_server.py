"""GPU tests of the server (pa_server_*): continuous admission, bit-exact results.

Each served result must equal the oracle and the same request hashed alone;
admission must respect the HBM budget and the slot count.
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


def _jobs(blocks):
    """Device requests; complete (synchronised) before they are submitted, as
    pa_server_submit requires of device keys without a ready event."""
    import torch
    jobs = [{"key": torch.from_numpy(b.key().view(np.int64)).cuda(),
             "out": torch.full((workloads.words(b.m),), -1, dtype=torch.int64, device="cuda"),
             "n": b.n, "m": b.m, "seed_a": b.seed_a, "seed_b": b.seed_b} for b in blocks]
    torch.cuda.synchronize()
    return jobs


def _host(t):
    return t.cpu().numpy().view(np.uint64).copy()


def _alone(pa, blocks, jobs):
    import torch
    ctx = pa.pa_init(0)
    try:
        pa.pa_reserve(ctx, max(b.n for b in blocks))
        outs = []
        for b, j in zip(blocks, jobs):
            o = torch.zeros_like(j["out"])
            pa.pa_hash_async(ctx, j["key"], b.seed_a, b.seed_b, b.n, b.m, o)
            outs.append(o)
        torch.cuda.synchronize()
        return [_host(o) for o in outs]
    finally:
        pa.pa_destroy(ctx)


def test_served_stream_matches_oracle_and_alone(pa):
    blocks, times = workloads.served_requests(21, 40, n_lo=1e3, n_hi=2e6, rate_per_s=20000.0)
    jobs = _jobs(blocks)
    with pa.Server(hbm_budget=1 << 30, slots=6, max_n=2_000_000) as srv:
        lat, st = srv.run_trace(jobs, times)
        stats = srv.stats()
    assert st == [pa.PA_OK] * len(blocks)
    assert stats["completed"] == len(blocks) and stats["failed"] == 0
    assert stats["peak_inflight"] > 1          # requests overlapped on the device
    alone = _alone(pa, blocks, jobs)
    for b, j, a in zip(blocks, jobs, alone):
        got = _host(j["out"])
        assert np.array_equal(got, a), (b.n, b.m)
        assert np.array_equal(got, oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m))
    assert all(x >= 0 for x in lat)


def test_host_memory_requests(pa):
    blocks, _ = workloads.served_requests(22, 12, n_lo=1e2, n_hi=5e5)
    outs = [np.zeros(workloads.words(b.m), dtype=np.uint64) for b in blocks]
    keys = [b.key() for b in blocks]
    with pa.Server(hbm_budget=256 << 20, slots=4, max_n=500_000) as srv:
        tickets = [srv.submit(k, b.seed_a, b.seed_b, b.n, b.m, o)
                   for k, b, o in zip(keys, blocks, outs)]
        for t in tickets:
            st, lat = srv.wait(t)
            assert st == pa.PA_OK and lat >= 0
    for b, k, o in zip(blocks, keys, outs):
        assert np.array_equal(o, oracle.pa_hash(k, b.seed_a, b.seed_b, b.n, b.m))


def test_ready_event_orders_a_key_still_being_written(pa):
    """Device keys produced by queued work on another stream: each request
    waits for the event recorded after its key's copy, so it hashes the final
    key (the copy is queued behind a long dummy kernel, so without the wait the
    server would read the old contents)."""
    import torch
    blocks, _ = workloads.served_requests(24, 6, n_lo=1e5, n_hi=2e6)
    producer = torch.cuda.Stream()
    src = [torch.from_numpy(b.key().view(np.int64)).pin_memory() for b in blocks]
    keys = [torch.zeros(workloads.words(b.n), dtype=torch.int64, device="cuda") for b in blocks]
    outs = [torch.full((workloads.words(b.m),), -1, dtype=torch.int64, device="cuda")
            for b in blocks]
    big = torch.ones((2048, 2048), device="cuda")
    torch.cuda.synchronize()
    with pa.Server(hbm_budget=1 << 30, slots=4, max_n=2_000_000) as srv:
        tickets = []
        with torch.cuda.stream(producer):
            for b, k, h, o in zip(blocks, keys, src, outs):
                for _ in range(20):
                    big = big @ big / 2048.0              # keeps the producer busy
                k.copy_(h, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(producer)
                tickets.append(srv.submit(k, b.seed_a, b.seed_b, b.n, b.m, o, ready=ev))
        for t in tickets:
            st, _ = srv.wait(t)
            assert st == pa.PA_OK
    torch.cuda.synchronize()
    for b, o in zip(blocks, outs):
        assert np.array_equal(_host(o), oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m))


def test_host_requests_through_run_trace(pa):
    """Open-loop replay of host-memory requests: every latency includes the
    key's copy to the device and the result's copy back; results equal the
    oracle."""
    blocks, times = workloads.served_requests(25, 16, n_lo=1e4, n_hi=1e6, rate_per_s=5000.0)
    jobs = [{"key": b.key(), "out": np.zeros(workloads.words(b.m), dtype=np.uint64), "n": b.n,
             "m": b.m, "seed_a": b.seed_a, "seed_b": b.seed_b} for b in blocks]
    with pa.Server(hbm_budget=512 << 20, slots=4, max_n=1_000_000) as srv:
        lat, st = srv.run_trace(jobs, times, device=False)
    assert st == [pa.PA_OK] * len(blocks)
    assert all(x > 0 for x in lat)
    for b, j in zip(blocks, jobs):
        assert np.array_equal(j["out"], oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m))


def test_admission_respects_budget(pa):
    # A budget that holds about two of the largest requests at a time.
    n_max = 3_000_000
    budget = 2 * pa.pa_workspace_bytes(n_max) + (8 << 20)
    blocks, times = workloads.served_requests(23, 24, n_lo=1e6, n_hi=n_max, rate_per_s=1e6)
    jobs = _jobs(blocks)
    with pa.Server(hbm_budget=budget, slots=8, max_n=n_max) as srv:
        lat, st = srv.run_trace(jobs, times)
        stats = srv.stats()
    assert st == [pa.PA_OK] * len(blocks)
    assert stats["peak_bytes"] <= budget
    assert 1 <= stats["peak_inflight"] <= 8
    alone = _alone(pa, blocks, jobs)
    for j, a in zip(jobs, alone):
        assert np.array_equal(_host(j["out"]), a)


def test_rejects_oversized_and_invalid(pa):
    import torch
    with pa.Server(hbm_budget=64 << 20, slots=2, max_n=100_000) as srv:
        key = torch.zeros(4000, dtype=torch.int64, device="cuda")
        out = torch.zeros(4000, dtype=torch.int64, device="cuda")
        for n, m in [(200_000, 10), (1000, 0), (1000, 1001)]:
            with pytest.raises(pa.PAError) as e:
                srv.submit(key, 1, 2, n, m, out)
            assert e.value.status == pa.PA_EINVAL
    with pytest.raises(pa.PAError):
        pa.Server(hbm_budget=1 << 20, slots=2, max_n=10**8)   # cannot hold one request


def test_served_workload_full_sizes(pa):
    """Requests of the served workload's sizes (n log-uniform in [1e6, 1e8],
    m = 0.3 n) arriving faster than they can be served: every result equals
    the lone result; the largest and two more are checked against the oracle."""
    blocks, times = workloads.served_requests(4, 48, rate_per_s=20000.0)
    _log(f"served: {sum(b.n for b in blocks)} bits, n max {max(b.n for b in blocks)}")
    jobs = _jobs(blocks)
    budget = 8 << 30
    with pa.Server(hbm_budget=budget, slots=8, max_n=10**8) as srv:
        lat, st = srv.run_trace(jobs, times)
        stats = srv.stats()
    assert st == [pa.PA_OK] * len(blocks)
    assert stats["peak_bytes"] <= budget and stats["peak_inflight"] > 1
    alone = _alone(pa, blocks, jobs)
    for j, a in zip(jobs, alone):
        assert np.array_equal(_host(j["out"]), a)
    order = sorted(range(len(blocks)), key=lambda i: -blocks[i].n)
    for i in [order[0], order[len(order) // 2], order[-1]]:
        b = blocks[i]
        _log(f"oracle check n={b.n}")
        assert np.array_equal(_host(jobs[i]["out"]),
                              oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m))


def test_waited_ticket_is_retired_and_explicit_operands_are_refused(pa):
    import torch
    blocks, _ = workloads.served_requests(24, 3, n_lo=1e3, n_hi=1e5)
    jobs = _jobs(blocks)
    with pa.Server(hbm_budget=64 << 20, slots=2, max_n=100_000) as srv:
        j, b = jobs[0], blocks[0]
        t = srv.submit(j["key"], b.seed_a, b.seed_b, b.n, b.m, j["out"])
        assert srv.wait(t)[0] == pa.PA_OK
        with pytest.raises(pa.PAError) as e:
            srv.wait(t)
        assert e.value.status == pa.PA_EINVAL
        # a trace job with an explicit operand is not submitted
        jobs[1]["c"] = torch.ones(workloads.words(blocks[1].n), dtype=torch.int64, device="cuda")
        lat, st = srv.run_trace(jobs[1:], [0.0, 0.0])
        assert st == [pa.PA_EINVAL, pa.PA_OK] and lat[0] == -1 and lat[1] >= 0
        srv.drain()
        stats = srv.stats()
    assert stats["completed"] == 2 and stats["failed"] == 0
    for b, j in zip(blocks[::2], jobs[::2]):
        assert np.array_equal(_host(j["out"]), oracle.pa_hash(b.key(), b.seed_a, b.seed_b, b.n, b.m))
