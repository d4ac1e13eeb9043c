"""Benchmark: G_{c,d} privacy-amplification hash throughput on one MI355X.

One step = one hash of a single n = 10^8-bit block (m = 4*10^7 output bits,
key / multiplier / addend uniform random from workload seed 2), run through the
device-resident entry point with the key already in HBM.  Prints one JSON line:
throughput in Mbps of input key, the roofline of the dominant kernel (timed with
HIP events on the stream it runs on), the CPU oracle timed on this host, and,
beside them, the n = 10^6 block, the 256-block batch (batched vs plain) and the
served stream (p50 / p99 latency at three offered loads).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PA Mbps (input bits/s) at n=1e6,1e8 bit-exact; batched vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0
PAPER_MBPS_N1E8 = 140.96   # Table 2, i9-9900k, n = 10^8 (m not stated)
COUNTERS = os.path.join(ROOT, "profiles", "counters_ntt_pass_n1e8.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # the clocks rise over the first ~60 n = 10^8 blocks (about 20 ms) of
    # sustained load; the default warm-up covers that
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="n1e8", choices=["n1e6", "n1e7", "n1e8"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-cpu-single-thread", action="store_true",
                    help="skip the oracle's single-thread leg (about 25 s at n = 10^8)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the n=1e6, batched and served measurements")
    ap.add_argument("--only-batch", action="store_true",
                    help="with --no-cpu: time only the 256-block batch (quick check)")
    ap.add_argument("--profile-runs", type=int, default=5)
    ap.add_argument("--served-requests", type=int, default=2000)
    ap.add_argument("--plan", default=None, metavar="T,TS,R0",
                    help="use this transform geometry for the main workload instead of "
                         "autotuning it (tile log, strided tile log, factor-3 rows log)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first stream this many MiB through a plain element-wise kernel "
                         "(bitwise_not, int64): the known-size reference for HBM counters")
    ap.add_argument("--ingest-counters", nargs="+", metavar="DIR",
                    help="no GPU: read rocprofv3 --pmc csv output under these directories "
                         "(FETCH_SIZE run, WRITE_SIZE run, optional SQ run) and write the "
                         "per-launch traffic of the NTT pass kernel to " +
                         os.path.relpath(COUNTERS, ROOT))
    return ap.parse_args()


def kernel_source_hash() -> str:
    """Hash of the pass kernel's code (comments and blank lines removed), so that
    committed counter readings are used only while they describe this code."""
    import re
    h = hashlib.sha256()
    for f in ("ntt.hip", "pass_body.h", "splitmix.h", "field.h", "kernels.h", "swizzle.h"):
        with open(os.path.join(ROOT, "paper_1910_04429_amd", "csrc", f)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update("\n".join(l.strip() for l in text.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from committed counter runs,
    or None when they are missing or were taken on other kernel source."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_hash") != kernel_source_hash():
        return None
    return c.get("bytes_per_launch")


VALU_ISSUE_LANE_OPS = 256 * 64 * 2.4e9   # one wave64 VALU instruction per CU per cycle


def valu_rate(avg_ms):
    """VALU issue of the dominant kernel: instructions from the committed SQ
    counter run x 64 lanes / live launch time, as a fraction of one wave64
    instruction per CU per cycle.  Not a hard ceiling: simple integer ops
    (v_add_u32) were measured issuing at 1.56x that rate and the 32-bit
    multiplies at 0.88-0.96x, so a fraction below 1 does not by itself show
    that the VALU is saturated.  None when the counters are stale."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_hash") != kernel_source_hash() or "SQ_INSTS_VALU" not in c.get("sq", {}):
        return None
    ops = c["sq"]["SQ_INSTS_VALU"] * 64 / (avg_ms * 1e-3)
    return {"lane_ops_per_s": ops, "one_instruction_per_cu_cycle": VALU_ISSUE_LANE_OPS,
            "issue_frac": round(ops / VALU_ISSUE_LANE_OPS, 4),
            "valu_insts_per_launch": c["sq"]["SQ_INSTS_VALU"],
            "note": "measured rates: v_add_u32 1.56x, v_mul_lo_u32 0.88x, v_mul_hi_u32 0.96x "
                    "of one instruction per CU-cycle"}


def _counter_rows(d):
    """(dispatch, kernel name, counter, value) from rocprofv3 csv files under d."""
    import csv
    rows = []
    for dirpath, _, files in os.walk(d):
        for fn in files:
            if not fn.endswith("counter_collection.csv"):
                continue
            with open(os.path.join(dirpath, fn)) as fh:
                for r in csv.DictReader(fh):
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"],
                                 float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    return rows


def _last_hashes(disps, hashes=3):
    """The k_pass values of the last `hashes` complete hashes: runs of k_pass
    dispatches that end at a carry kernel (one hash = one run)."""
    runs, cur = [], []
    for _, (name, v) in sorted(disps.items()):
        if "k_pass" in name:
            cur.append(v)
        elif "k_carry" in name and cur:
            runs.append(cur)
            cur = []
    runs = [r for r in runs if len(r) == len(runs[-1])] if runs else []
    return runs[-hashes:]


def ingest_counters(dirs, calib_mib, path=COUNTERS):
    """Per-launch HBM traffic of k_pass from FETCH_SIZE / WRITE_SIZE runs (KiB per
    dispatch), each scaled by what the same counter reads for the calibration
    kernel, which reads and writes exactly calib_mib MiB.  Only the k_pass
    launches of the last three hashes count (the end of the timed steps and the
    per-launch profile, all on one geometry)."""
    known_kib = calib_mib * 1024.0
    out = {"kernel": "k_pass", "workload": "n1e8", "source_hash": kernel_source_hash(),
           "calibration": {"kernel": "bitwise_not on int64 (reads and writes the given size)",
                           "mib": calib_mib}, "sq": {}}
    per = {}
    for d in dirs:
        per_counter = {}
        for disp, name, counter, val in _counter_rows(d):
            per_counter.setdefault(counter, {}).setdefault(disp, [name, 0.0])[1] += val
        for counter, disps in per_counter.items():
            hashes = _last_hashes(disps)
            cal = [v for _, (nm, v) in sorted(disps.items()) if "bitwise_not" in nm]
            per[counter] = {"hashes": hashes, "calib": cal}
    npass = None
    for counter, key in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        if counter not in per:
            raise SystemExit(f"{counter} missing from {dirs}")
        hashes, cal = per[counter]["hashes"], per[counter]["calib"]
        if not hashes or not cal:
            raise SystemExit(f"{counter}: no k_pass hashes or calibration dispatches")
        npass = len(hashes[0])
        factor = known_kib / float(np.median(cal))
        flat = [v for h in hashes for v in h]
        out["calibration"][f"{key}_kib_read"] = float(np.median(cal))
        out["calibration"][f"{key}_factor"] = round(factor, 4)
        out[f"{key}_kib_per_launch"] = float(np.mean(flat))
        out[f"{key}_bytes_per_launch"] = float(np.mean(flat)) * 1024 * factor
        out[f"{key}_kib_per_pass"] = [float(np.median([h[i] for h in hashes])) for i in range(npass)]
    out["passes_per_hash"] = npass
    out["sq_per_pass"] = {}
    for counter, v in per.items():
        if counter.startswith("SQ_") or counter.startswith("GRBM_"):
            flat = [x for h in v["hashes"] for x in h]
            out["sq"][counter] = float(np.mean(flat)) if flat else None
            if v["hashes"]:
                n = len(v["hashes"][0])
                out["sq_per_pass"][counter] = [float(np.median([h[i] for h in v["hashes"]]))
                                               for i in range(n)]
    out["bytes_per_launch"] = int(out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"])
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
    return out


def progress(msg):
    """One line per finished phase on stderr (the JSON line is the only stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(blk, key, single_thread=True):
    """The oracle on the whole n = 10^8 block on this host: once with its
    Karatsuba's top three levels split over 27 threads (at least one per
    logical CPU of a 16-CPU host), once on one thread.  A reported baseline,
    not a target: a Karatsuba low product, not GMP."""
    import oracle
    ncpu = os.cpu_count() or 1
    levels = 3                       # 3^3 = 27 threads
    threads = 3 ** levels
    t0 = time.perf_counter()
    y = oracle.pa_hash(key, blk.seed_a, blk.seed_b, blk.n, blk.m, par_levels=levels)
    dt = time.perf_counter() - t0
    res = {"value": blk.n / dt / 1e6, "unit": "Mbps", "cores": min(threads, ncpu),
           "threads": threads, "kind": "oracle", "cpu": cpu_model(), "host_logical_cpus": ncpu,
           "sample": f"one full block n={blk.n} m={blk.m} ({dt:.2f} s), Karatsuba low product "
                     f"with its top {levels} levels on {threads} threads over the host's "
                     f"{ncpu} logical CPUs"}
    if single_thread:
        t0 = time.perf_counter()
        y1 = oracle.pa_hash(key, blk.seed_a, blk.seed_b, blk.n, blk.m, par_levels=0)
        dt1 = time.perf_counter() - t0
        assert np.array_equal(y1, y), "the oracle's threaded and single-thread results differ"
        res["single_thread"] = {"value": blk.n / dt1 / 1e6, "unit": "Mbps", "cores": 1,
                                "sample": f"the same block on one thread ({dt1:.2f} s)"}
    return y, res


def time_single(pa, ctx, torch, blk, steps, warmup, plan=None):
    """ms per block for one block through pa_hash_async, key resident (the
    context's transform geometry for this length is autotuned first, unless
    a plan is given; the key is uploaded before, so that the warm-up follows
    the tuner's device work without a pause)."""
    d_key = torch.from_numpy(blk.key().view(np.int64)).cuda()
    d_out = torch.zeros(pa.words(blk.m), dtype=torch.int64, device="cuda")
    pa.pa_reserve(ctx, blk.n)
    torch.cuda.synchronize()
    if plan is None:
        pa.pa_tune(ctx, blk.n, 8)
    else:
        pa.pa_plan_set(ctx, blk.n, plan)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        pa.pa_hash_async(ctx, d_key, blk.seed_a, blk.seed_b, blk.n, blk.m, d_out, stream)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record(stream)
    for _ in range(steps):
        pa.pa_hash_async(ctx, d_key, blk.seed_a, blk.seed_b, blk.n, blk.m, d_out, stream)
    e.record(stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps, d_key, d_out


def per_block_latency(pa, ctx, torch, blk, d_key, d_out, runs=50):
    """Median and p99 of single blocks, each bracketed by its own events."""
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(runs)]
    for s, e in ev:
        s.record(stream)
        pa.pa_hash_async(ctx, d_key, blk.seed_a, blk.seed_b, blk.n, blk.m, d_out, stream)
        e.record(stream)
    torch.cuda.synchronize()
    ms = np.array([s.elapsed_time(e) for s, e in ev])
    return {"median_ms": round(float(np.median(ms)), 4),
            "p99_ms": round(float(np.percentile(ms, 99)), 4), "runs": runs}


def copy_bandwidth(torch, mib=1024, reps=10):
    """Device-to-device copy rate (bytes read + written per second) of a
    1 GiB buffer: the practical HBM ceiling next to the 8 TB/s spec."""
    src = torch.zeros(mib << 17, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        dst.copy_(src)
    e.record()
    torch.cuda.synchronize()
    gbs = 2 * src.numel() * 8 * reps / (s.elapsed_time(e) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def host_to_host(pa, ctx, blk, key):
    """pa_hash from pageable host memory to host memory: the PCIe-inclusive rate
    (context only; the reported value keeps the key resident in HBM)."""
    for _ in range(2):
        pa.pa_hash(ctx, key, blk.seed_a, blk.seed_b, blk.n, blk.m)
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        pa.pa_hash(ctx, key, blk.seed_a, blk.seed_b, blk.n, blk.m)
    ms = (time.perf_counter() - t0) / reps * 1e3
    return {"ms_per_block": round(ms, 3), "mbps": round(blk.n / (ms * 1e-3) / 1e6, 1),
            "note": "pa_hash: key in and result out through pageable host memory"}


def toeplitz_rate(pa, ctx, torch, blk, reps):
    """The Toeplitz-hash variant on the same block (t from seed_a): ms and Mbps."""
    d_key = torch.from_numpy(blk.key().view(np.int64)).cuda()
    d_out = torch.zeros(pa.words(blk.m), dtype=torch.int64, device="cuda")
    for _ in range(2):
        pa.pa_toeplitz_async(ctx, d_key, None, blk.seed_a, blk.n, blk.m, d_out)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        pa.pa_toeplitz_async(ctx, d_key, None, blk.seed_a, blk.n, blk.m, d_out)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    L, pieces = pa.pa_toeplitz_length(blk.n, blk.m)
    return {"ms_per_block": round(ms, 4), "mbps": round(blk.n / (ms * 1e-3) / 1e6, 1),
            "transform_length": L, "key_pieces": pieces}


def cached_multiplier(pa, ctx, torch, blk, d_key):
    """Opt-in mode: the multiplier's transform computed once and reused, so a
    block costs two transforms instead of three.  Not the headline value."""
    mul = pa.pa_mul_create(ctx, blk.seed_a, blk.n)
    d_out = torch.zeros(pa.words(blk.m), dtype=torch.int64, device="cuda")
    try:
        for _ in range(3):
            pa.pa_hash_mul_async(ctx, mul, d_key, blk.seed_b, blk.n, blk.m, d_out)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(20):
            pa.pa_hash_mul_async(ctx, mul, d_key, blk.seed_b, blk.n, blk.m, d_out)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / 20
    finally:
        pa.pa_mul_destroy(mul)
    return {"ms_per_block": round(ms, 4), "mbps": round(blk.n / (ms * 1e-3) / 1e6, 1),
            "note": "multiplier transform cached across blocks (opt-in pa_mul_*)"}


def batched_vs_plain(pa, ctx, torch, workloads):
    """256 blocks, n log-uniform in [1e5, 1e7]: the grouped launches (captured
    into a HIP graph and replayed) against the same blocks hashed one at a time."""
    blocks = workloads.batch_blocks(3, 256)
    bits = sum(b.n for b in blocks)
    jobs = [{"key": torch.from_numpy(b.key().view(np.int64)).cuda(),
             "out": torch.zeros(workloads.words(b.m), dtype=torch.int64, device="cuda"),
             "n": b.n, "m": b.m, "seed_a": b.seed_a, "seed_b": b.seed_b} for b in blocks]
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"workload": "256 blocks, n log-uniform in [1e5, 1e7], m = round(r n), "
                       "r uniform in [0.05, 0.5], seed 3", "bits": bits}
    for name, tune in (("grouped", False), ("grouped_tuned", True)):
        batch = pa.Batch(ctx, jobs, mode=pa.PA_BATCH_GROUPED)
        try:
            if tune:
                batch.tune(3)
                res["tuned_groups"] = batch.groups()
            batch.capture()
            for _ in range(3):
                batch.run()
            torch.cuda.synchronize()
            s.record()
            reps = 10
            for _ in range(reps):
                batch.run()
            e.record()
            torch.cuda.synchronize()
            if batch.result() != pa.PA_OK:
                raise RuntimeError(f"{name} batch run reported a failure")
            ms = s.elapsed_time(e) / reps
            res[name] = {"ms": round(ms, 3), "mbps": round(bits / (ms * 1e-3) / 1e6, 1),
                         "launches_per_run": batch.launches()}
        finally:
            batch.close()
    res["grouped"]["runs"] = "one launch per pass per length group, groups on 4 streams, captured HIP graph"
    res["grouped_tuned"]["runs"] = "the same after pa_batch_tune (geometry per length group, measured)"
    res["persistent"] = "not run: the persistent queue kernel is switched off (not yet validated on a GPU)"
    pa.pa_reserve(ctx, max(b.n for b in blocks))
    for b, j in zip(blocks, jobs):
        pa.pa_hash_async(ctx, j["key"], b.seed_a, b.seed_b, b.n, b.m, j["out"])
    torch.cuda.synchronize()
    s.record()
    for b, j in zip(blocks, jobs):
        pa.pa_hash_async(ctx, j["key"], b.seed_a, b.seed_b, b.n, b.m, j["out"])
    e.record()
    torch.cuda.synchronize()
    ms_plain = s.elapsed_time(e)
    res["plain"] = {"ms": round(ms_plain, 3), "mbps": round(bits / (ms_plain * 1e-3) / 1e6, 1),
                    "runs": "pa_hash_async per block, one stream"}
    return res


def served(pa, torch, workloads, count):
    """Poisson stream of requests, n log-uniform in [1e6, 1e8], m = 0.3 n.
    Device-resident requests: saturated throughput C first (all requests at
    t = 0), then offered loads rho C for rho in (0.5, 0.8, 0.95).  Then the same
    requests from host memory (each latency includes the key's copy to the
    device and the result's copy back): their own saturated throughput and the
    same three loads of it.  Each request's key is its own window of one
    seeded pool of 2^25 words (the hash does the same work on any key bits)."""
    blocks, unit_times = workloads.served_requests(4, count, rate_per_s=1.0)
    pool_words = 1 << 25
    pool_host = workloads.key_bits(workloads.seeds_of(4)[0], 64 * pool_words)
    rng = np.random.default_rng(4)
    # even word offsets keep every key 16-byte aligned, as a fresh allocation is
    offs = [2 * int(rng.integers(0, (pool_words - workloads.words(b.n)) // 2 + 1)) for b in blocks]
    pool = torch.from_numpy(pool_host.view(np.int64)).cuda()
    dev_jobs = [{"key": pool[o: o + workloads.words(b.n)],
                 "out": torch.zeros(workloads.words(b.m), dtype=torch.int64, device="cuda"),
                 "n": b.n, "m": b.m, "seed_a": b.seed_a, "seed_b": b.seed_b}
                for b, o in zip(blocks, offs)]
    host_jobs = [{"key": pool_host[o: o + workloads.words(b.n)],
                  "out": np.zeros(workloads.words(b.m), dtype=np.uint64),
                  "n": b.n, "m": b.m, "seed_a": b.seed_a, "seed_b": b.seed_b}
                 for b, o in zip(blocks, offs)]
    torch.cuda.synchronize()
    mean_n = sum(b.n for b in blocks) / len(blocks)
    budget = 16 << 30
    res = {"workload": f"{count} requests, n log-uniform in [1e6, 1e8], m = 0.3 n, "
                       "Poisson arrivals, seed 4; each key a window of a seeded 2^31-bit pool, "
                       "seeds per request",
           "hbm_budget_bytes": budget, "slots": 8}

    def run(jobs, device):
        out = {"loads": []}
        with pa.Server(hbm_budget=budget, slots=8, max_n=10**8) as srv:
            srv.run_trace(jobs[:64], [0.0] * 64, device=device)          # warm-up
        with pa.Server(hbm_budget=budget, slots=8, max_n=10**8) as srv:
            srv.run_trace(jobs, [0.0] * len(jobs), device=device)
            sat = srv.stats()
        C = sat["bits"] / sat["wall_s"]
        out["saturated_mbps"] = round(C / 1e6, 1)
        for rho in (0.5, 0.8, 0.95):
            rate = rho * C / mean_n                                     # requests per second
            times = np.asarray(unit_times) / rate
            with pa.Server(hbm_budget=budget, slots=8, max_n=10**8) as srv:
                lat, st = srv.run_trace(jobs, times, device=device)
                s = srv.stats()
            out["loads"].append({"rho": rho, "offered_mbps": round(rho * C / 1e6, 1),
                                 "mbps": round(s["bits"] / s["wall_s"] / 1e6, 1),
                                 "p50_ms": round(s["lat_p50_ms"], 3),
                                 "p99_ms": round(s["lat_p99_ms"], 3),
                                 "mean_ms": round(s["lat_mean_ms"], 3),
                                 "peak_inflight": s["peak_inflight"],
                                 "all_ok": all(x == pa.PA_OK for x in st)})
        return out

    dev = run(dev_jobs, True)
    res["saturated_mbps"] = dev["saturated_mbps"]
    res["loads"] = dev["loads"]
    res["host_data"] = run(host_jobs, False)
    res["host_data"]["note"] = ("key and result in host memory: latency from arrival to the "
                                "result in host memory, copies included")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library "
              "hashes each block on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.ingest_counters:
        ingest_counters(args.ingest_counters, args.copy_calibration_mib or 256)
        return

    import torch
    import paper_1910_04429_amd as pa
    import workloads

    blk = workloads.single(args.workload)
    key = blk.key()
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        src = torch.zeros(args.copy_calibration_mib << 17, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ctx = pa.pa_init(0)
    t0 = time.perf_counter()
    plan = None
    if args.plan:
        t, ts, r0 = (int(v) for v in args.plan.split(","))
        plan = {"tile_log": t, "strided_tile_log": ts, "rows3_log": r0}
    ms_per_step, d_key, d_out = time_single(pa, ctx, torch, blk, args.steps, args.warmup, plan)
    wall = time.perf_counter() - t0
    progress(f"{args.workload}: {ms_per_step:.4f} ms per step")
    mbps = blk.n / (ms_per_step * 1e-3) / 1e6
    latency = per_block_latency(pa, ctx, torch, blk, d_key, d_out)
    gpu_out = d_out.cpu().numpy().view(np.uint64).copy()

    # per-launch HIP events, same stream, outside the timed region
    stream = torch.cuda.current_stream()
    kinds = {}
    for _ in range(args.profile_runs):
        for rec in pa.pa_hash_profile(ctx, d_key, blk.seed_a, blk.seed_b, blk.n, blk.m,
                                      d_out, stream):
            k = kinds.setdefault(rec["kind"], {"ms": 0.0, "bytes": 0, "launches": 0})
            k["ms"] += rec["ms"]
            k["bytes"] += rec["bytes"]
            k["launches"] += 1
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    d = kinds[dom]
    avg_ms = d["ms"] / d["launches"]
    avg_bytes = d["bytes"] / d["launches"]
    achieved = avg_bytes / (avg_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "kernel": f"k_pass ({dom})", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic() if args.workload == "n1e8" else None,
                "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": int(avg_bytes),
                "valu_issue": valu_rate(avg_ms) if args.workload == "n1e8" else None}
    copy_gbs = copy_bandwidth(torch)
    roofline["measured_copy_gbs"] = copy_gbs
    roofline["frac_of_measured_copy"] = round(achieved / copy_gbs, 4)
    breakdown = {k: {"ms_per_step": round(v["ms"] / args.profile_runs, 4),
                     "launches_per_step": v["launches"] // args.profile_runs}
                 for k, v in kinds.items()}

    extra = {}
    if args.only_batch:
        print(json.dumps(batched_vs_plain(pa, ctx, torch, workloads)), flush=True)
        pa.pa_destroy(ctx)
        return
    if not args.no_extra:
        progress("extras: n1e6, n1e7, host-to-host, cached multiplier, Toeplitz, batch, served")
        b6 = workloads.single("n1e6")
        ms6, _, _ = time_single(pa, ctx, torch, b6, 200, 500)
        extra["n1e6"] = {"ms_per_block": round(ms6, 4), "mbps": round(b6.n / (ms6 * 1e-3) / 1e6, 1),
                         "paper_mbps_i9": 262.13}
        b7 = workloads.single("n1e7")
        ms7, _, _ = time_single(pa, ctx, torch, b7, 100, 250)
        extra["n1e7"] = {"ms_per_block": round(ms7, 4), "mbps": round(b7.n / (ms7 * 1e-3) / 1e6, 1),
                         "paper_mbps_i9": 187.86}
        extra["n1e8_host_to_host"] = host_to_host(pa, ctx, blk, key)
        extra["n1e8_cached_multiplier"] = cached_multiplier(pa, ctx, torch, blk, d_key)
        extra["toeplitz"] = {
            "note": "Toeplitz-hash variant (GF(2) Toeplitz matrix, t of n+m-1 bits) on the "
                    "same transform engine, one element per key bit over one prime",
            "n1e6": toeplitz_rate(pa, ctx, torch, workloads.single("n1e6"), 50),
            "n1e8": toeplitz_rate(pa, ctx, torch, blk, 5)}
        extra["batched"] = batched_vs_plain(pa, ctx, torch, workloads)
        progress("batch done")
        extra["served"] = served(pa, torch, workloads, args.served_requests)
        progress("served done")

    cpu = None
    bit_exact = None
    if not args.no_cpu:
        progress("CPU oracle")
        want, cpu = cpu_baseline(blk, key, not args.no_cpu_single_thread)
        bit_exact = bool(np.array_equal(gpu_out, want))

    plan = pa.pa_plan_get(ctx, blk.n)
    plan.pop("ms", None)
    plan["chosen_by"] = "given (--plan)" if args.plan else "pa_tune"
    pa.pa_destroy(ctx)
    vs = mbps / PAPER_MBPS_N1E8 if args.workload == "n1e8" else None
    line = {
        "metric": METRIC, "value": round(mbps, 1), "unit": "Mbps", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(vs, 1) if vs else None,
        "baseline_ref": "paper Table 2, i9-9900k CPU, n=1e8: 140.96 Mbps (other hardware; context)",
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"single PA block {args.workload}: n={blk.n} m={blk.m} "
                               f"uniform random key/c/d from seed "
                               f"{workloads.SINGLE_BLOCKS[args.workload][2]}",
                   "n": blk.n, "m": blk.m, "transform_length": pa.pa_transform_length(blk.n),
                   "plan": plan},
        "per_block": latency,
        "bit_exact_vs_oracle": bit_exact,
        "roofline": roofline,
        "kernels": breakdown,
        "cpu_baseline": cpu,
        **extra,
        "host_wall_s_timed_region": round(wall, 4),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
