"""Python binding of libpa, the G_{c,d} privacy-amplification hash on MI355X.

Thin ctypes marshalling over the C ABI declared in include/pa.h; every step of
the hash runs in the library's HIP kernels.  The functions keep the C names:

    ctx = pa_init(device=0)
    y = pa_hash(ctx, key_words, seed_a, seed_b, n, m)          # host in/out
    y = pa_hash_ex(ctx, key_words, c_words, d_words, n, m)     # explicit c, d
    pa_hash_async(ctx, d_key, seed_a, seed_b, n, m, d_out)     # torch device tensors
    prof = pa_hash_profile(ctx, d_key, seed_a, seed_b, n, m, d_out)
    pa_destroy(ctx)

Host arrays are numpy uint64 (little-endian words, bit i of the value at bit
i % 64 of word i // 64).  Device buffers are torch tensors of 8-byte elements on
a ROCm device; torch only provides their memory and the HIP stream.

The library is built in-tree (``python -m paper_1910_04429_amd.build`` or
``__graft_entry__.build()``).  If libpa.so is missing this module raises at
import: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpa.so")

PA_OK, PA_EINVAL, PA_ENOMEM, PA_EDEVICE, PA_ENODEV, PA_EIO = 0, 1, 2, 3, 4, 5
PA_MAX_N = 1 << 29
PA_TOEPLITZ_MAX_M = 3 << 24
PA_PROFILE_MAX = 32
PA_NOALLOC_MAX_BYTES = 120 << 20
KERNEL_KINDS = {0: "ntt_pass", 1: "carry_local", 3: "carry_apply"}


class PAError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"libpa status {status}: {text}")
        self.status = status


class _Profile(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int),
                ("kind", ctypes.c_int * PA_PROFILE_MAX),
                ("ms", ctypes.c_float * PA_PROFILE_MAX),
                ("bytes", ctypes.c_uint64 * PA_PROFILE_MAX)]


class _Job(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("c", ctypes.c_void_p), ("d", ctypes.c_void_p),
                ("seed_a", ctypes.c_uint64), ("seed_b", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("out", ctypes.c_void_p), ("status", ctypes.c_int)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("wait_us", ctypes.c_uint32),
                ("force_abort", ctypes.c_int)]


PA_BATCH_PERSISTENT, PA_BATCH_GROUPED = 0, 1


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("slots", ctypes.c_int),
                ("max_n", ctypes.c_uint64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("bits", ctypes.c_uint64), ("peak_inflight", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("lat_p50_ms", ctypes.c_double),
                ("lat_p99_ms", ctypes.c_double), ("lat_mean_ms", ctypes.c_double),
                ("wall_s", ctypes.c_double)]


PA_SUBMIT_DEVICE = 1

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u64 = ctypes.c_uint64

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")

# libpa needs the HIP runtime by its soname (libamdhip64.so.7).  torch ships its
# own copy under the same soname; loading torch first makes the dynamic linker
# bind libpa to that one, so the process has a single HIP runtime and torch's
# device pointers and streams are valid inside libpa.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

class _Opts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("tune_cache", ctypes.c_char_p)]


_lib.pa_init.restype = ctypes.c_int
_lib.pa_init.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(_Opts)]
_lib.pa_ctx_bytes.restype = ctypes.c_uint64
_lib.pa_ctx_bytes.argtypes = [ctypes.c_void_p]
_lib.pa_destroy.restype = None
_lib.pa_destroy.argtypes = [ctypes.c_void_p]
_lib.pa_strerror.restype = ctypes.c_char_p
_lib.pa_strerror.argtypes = [ctypes.c_int]
_lib.pa_last_error.restype = ctypes.c_char_p
_lib.pa_last_error.argtypes = [ctypes.c_void_p]
_lib.pa_hash.restype = ctypes.c_int
_lib.pa_hash.argtypes = [ctypes.c_void_p, _u64p, _u64, _u64, _u64, _u64, _u64p]
_lib.pa_hash_ex.restype = ctypes.c_int
_lib.pa_hash_ex.argtypes = [ctypes.c_void_p, _u64p, _u64p, _u64p, _u64, _u64, _u64p]
_lib.pa_hash_async.restype = ctypes.c_int
_lib.pa_hash_async.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _u64, _u64, _u64, _u64,
                               ctypes.c_void_p, ctypes.c_void_p]
_lib.pa_hash_async_noalloc.restype = ctypes.c_int
_lib.pa_hash_async_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _u64, _u64, _u64, _u64,
                                       ctypes.c_void_p, ctypes.c_void_p]
_lib.pa_hash_profile.restype = ctypes.c_int
_lib.pa_hash_profile.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _u64, _u64, _u64, _u64,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Profile)]
_lib.pa_reserve.restype = ctypes.c_int
_lib.pa_reserve.argtypes = [ctypes.c_void_p, _u64]
_lib.pa_workspace_bytes.restype = _u64
_lib.pa_workspace_bytes.argtypes = [_u64]
_lib.pa_transform_length.restype = _u64
_lib.pa_transform_length.argtypes = [_u64]
class _Plan(ctypes.Structure):
    _fields_ = [("tile_log", ctypes.c_int), ("strided_tile_log", ctypes.c_int),
                ("rows3_log", ctypes.c_int), ("passes", ctypes.c_int), ("ms", ctypes.c_float)]


_lib.pa_plan_candidates.restype = ctypes.c_int
_lib.pa_plan_candidates.argtypes = [_u64, ctypes.POINTER(_Plan), ctypes.c_int]
_lib.pa_plan_get.restype = ctypes.c_int
_lib.pa_plan_get.argtypes = [ctypes.c_void_p, _u64, ctypes.POINTER(_Plan)]
_lib.pa_plan_set.restype = ctypes.c_int
_lib.pa_plan_set.argtypes = [ctypes.c_void_p, _u64, ctypes.POINTER(_Plan)]
_lib.pa_tune.restype = ctypes.c_int
_lib.pa_tune.argtypes = [ctypes.c_void_p, _u64, ctypes.c_int, ctypes.POINTER(_Plan)]
_lib.pa_toeplitz.restype = ctypes.c_int
_lib.pa_toeplitz.argtypes = [ctypes.c_void_p, _u64p, _u64p, _u64, _u64, _u64, _u64p]
_lib.pa_toeplitz_async.restype = ctypes.c_int
_lib.pa_toeplitz_async.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _u64, _u64,
                                   _u64, ctypes.c_void_p, ctypes.c_void_p]
_lib.pa_toeplitz_length.restype = _u64
_lib.pa_toeplitz_length.argtypes = [_u64, _u64, ctypes.POINTER(_u64)]
_lib.pa_batch_create.restype = ctypes.c_int
_lib.pa_batch_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Job), ctypes.c_size_t,
                                 ctypes.POINTER(ctypes.c_void_p)]
_lib.pa_batch_create_ex.restype = ctypes.c_int
_lib.pa_batch_create_ex.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Job), ctypes.c_size_t,
                                    ctypes.POINTER(_BatchOpts), ctypes.POINTER(ctypes.c_void_p)]
_lib.pa_batch_result.restype = ctypes.c_int
_lib.pa_batch_result.argtypes = [ctypes.c_void_p]
_lib.pa_batch_run.restype = ctypes.c_int
_lib.pa_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.pa_batch_capture.restype = ctypes.c_int
_lib.pa_batch_capture.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.pa_batch_bytes.restype = _u64
_lib.pa_batch_bytes.argtypes = [ctypes.c_void_p]
_lib.pa_batch_size.restype = ctypes.c_size_t
_lib.pa_batch_size.argtypes = [ctypes.c_void_p]
_lib.pa_batch_launches.restype = ctypes.c_size_t
_lib.pa_batch_launches.argtypes = [ctypes.c_void_p]
_lib.pa_batch_destroy.restype = None
_lib.pa_batch_destroy.argtypes = [ctypes.c_void_p]
_lib.pa_batch_tune.restype = ctypes.c_int
_lib.pa_batch_tune.argtypes = [ctypes.c_void_p, ctypes.c_int]
_lib.pa_batch_groups.restype = ctypes.c_size_t
_lib.pa_batch_groups.argtypes = [ctypes.c_void_p]
_lib.pa_batch_group.restype = ctypes.c_int
_lib.pa_batch_group.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(ctypes.c_uint32), ctypes.c_void_p]
_lib.pa_hash_many.restype = ctypes.c_int
_lib.pa_hash_many.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Job), ctypes.c_size_t,
                              ctypes.c_void_p]

_lib.pa_server_create.restype = ctypes.c_int
_lib.pa_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(_ServerOpts),
                                  ctypes.POINTER(ctypes.c_void_p)]
_lib.pa_server_submit.restype = ctypes.c_int
_lib.pa_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _u64, _u64, _u64, _u64,
                                  ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
_lib.pa_server_submit_after.restype = ctypes.c_int
_lib.pa_server_submit_after.argtypes = [ctypes.c_void_p, ctypes.c_void_p, _u64, _u64, _u64, _u64,
                                        ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_uint64)]
_lib.pa_server_wait.restype = ctypes.c_int
_lib.pa_server_wait.argtypes = [ctypes.c_void_p, _u64, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_double)]
_lib.pa_server_drain.restype = ctypes.c_int
_lib.pa_server_drain.argtypes = [ctypes.c_void_p]
_lib.pa_server_get_stats.restype = ctypes.c_int
_lib.pa_server_get_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(_ServerStats)]
_lib.pa_server_run_trace.restype = ctypes.c_int
_lib.pa_server_run_trace.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Job),
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_size_t,
                                     ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int)]
_lib.pa_server_destroy.restype = None
_lib.pa_server_destroy.argtypes = [ctypes.c_void_p]

_lib.pa_mul_create.restype = ctypes.c_int
_lib.pa_mul_create.argtypes = [ctypes.c_void_p, _u64, ctypes.c_void_p, _u64, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]
_lib.pa_hash_mul_async.restype = ctypes.c_int
_lib.pa_hash_mul_async.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _u64, _u64,
                                   ctypes.c_void_p, ctypes.c_void_p]
_lib.pa_mul_destroy.restype = None
_lib.pa_mul_destroy.argtypes = [ctypes.c_void_p]

MASK64 = (1 << 64) - 1


def words(bits: int) -> int:
    return (int(bits) + 63) // 64


def _check(ctx, rc: int):
    if rc != PA_OK:
        detail = _lib.pa_last_error(ctx).decode() if ctx else ""
        raise PAError(rc, f"{_lib.pa_strerror(rc).decode()} {detail}".strip())


def _host_words(a, nwords: int, name: str) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    if a.ndim != 1 or a.size < nwords:
        raise ValueError(f"{name}: need {nwords} uint64 words, got shape {a.shape}")
    return a


def _dev_ptr(t, nwords: int, name: str) -> int:
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous() or t.element_size() != 8 or t.numel() < nwords:
        raise ValueError(f"{name}: need a contiguous 8-byte tensor of >= {nwords} elements")
    return t.data_ptr()


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def pa_init(device: int = 0, hbm_budget: int = 0, tune_cache: str | None = None):
    """A context on `device`; hbm_budget bounds the device bytes it holds (0:
    none), tune_cache names the file of tuned geometries (None: no file)."""
    ctx = ctypes.c_void_p()
    opts = _Opts(int(hbm_budget), tune_cache.encode() if tune_cache else None)
    _check(None, _lib.pa_init(ctypes.byref(ctx), int(device), ctypes.byref(opts)))
    return ctx


def pa_ctx_bytes(ctx) -> int:
    return int(_lib.pa_ctx_bytes(ctx))


def pa_destroy(ctx) -> None:
    if ctx:
        _lib.pa_destroy(ctx)


def pa_strerror(status: int) -> str:
    return _lib.pa_strerror(status).decode()


def pa_last_error(ctx) -> str:
    return _lib.pa_last_error(ctx).decode()


def pa_hash(ctx, key, seed_a: int, seed_b: int, n: int, m: int) -> np.ndarray:
    key = _host_words(key, words(n), "key")
    out = np.zeros(max(words(m), 1), dtype=np.uint64)
    _check(ctx, _lib.pa_hash(ctx, key.ctypes.data_as(_u64p), seed_a & MASK64,
                             seed_b & MASK64, n, m, out.ctypes.data_as(_u64p)))
    return out


def pa_hash_ex(ctx, key, c, d, n: int, m: int) -> np.ndarray:
    w = words(n)
    key, c, d = _host_words(key, w, "key"), _host_words(c, w, "c"), _host_words(d, w, "d")
    out = np.zeros(max(words(m), 1), dtype=np.uint64)
    _check(ctx, _lib.pa_hash_ex(ctx, key.ctypes.data_as(_u64p), c.ctypes.data_as(_u64p),
                                d.ctypes.data_as(_u64p), n, m, out.ctypes.data_as(_u64p)))
    return out


def pa_hash_async(ctx, d_key, seed_a: int, seed_b: int, n: int, m: int, d_out,
                  stream=None) -> None:
    """Queue the hash of device tensor d_key into device tensor d_out."""
    _check(ctx, _lib.pa_hash_async(ctx, _dev_ptr(d_key, words(n), "d_key"), seed_a & MASK64,
                                   seed_b & MASK64, n, m, _dev_ptr(d_out, words(m), "d_out"),
                                   _stream_handle(stream)))


def pa_hash_async_noalloc(ctx, d_key, seed_a: int, seed_b: int, n: int, m: int, d_out,
                          stream=None) -> None:
    """pa_hash_async without any device allocation: the block's working memory
    is the library's fixed per-GPU scratch (calls overlapping on one GPU race)."""
    _check(ctx, _lib.pa_hash_async_noalloc(ctx, _dev_ptr(d_key, words(n), "d_key"),
                                           seed_a & MASK64, seed_b & MASK64, n, m,
                                           _dev_ptr(d_out, words(m), "d_out"),
                                           _stream_handle(stream)))


def pa_hash_profile(ctx, d_key, seed_a: int, seed_b: int, n: int, m: int, d_out,
                    stream=None) -> list[dict]:
    """Run once with a HIP event pair around every launch; returns one dict per launch."""
    prof = _Profile()
    _check(ctx, _lib.pa_hash_profile(ctx, _dev_ptr(d_key, words(n), "d_key"),
                                     seed_a & MASK64, seed_b & MASK64, n, m,
                                     _dev_ptr(d_out, words(m), "d_out"),
                                     _stream_handle(stream), ctypes.byref(prof)))
    return [{"kind": KERNEL_KINDS.get(prof.kind[i], str(prof.kind[i])),
             "ms": float(prof.ms[i]), "bytes": int(prof.bytes[i])}
            for i in range(prof.count)]


def pa_mul_create(ctx, seed_a: int, n: int, c=None, stream=None):
    """Transform the multiplier once (opt-in reuse across blocks of n bits)."""
    h = ctypes.c_void_p()
    cp = _dev_ptr(c, words(n), "c") if c is not None else None
    _check(ctx, _lib.pa_mul_create(ctx, seed_a & MASK64, cp, n, _stream_handle(stream),
                                   ctypes.byref(h)))
    return h


def pa_hash_mul_async(ctx, mul, d_key, seed_b: int, n: int, m: int, d_out, stream=None) -> None:
    _check(ctx, _lib.pa_hash_mul_async(ctx, mul, _dev_ptr(d_key, words(n), "d_key"),
                                       seed_b & MASK64, m, _dev_ptr(d_out, words(m), "d_out"),
                                       _stream_handle(stream)))


def pa_mul_destroy(mul) -> None:
    if mul:
        _lib.pa_mul_destroy(mul)


def pa_reserve(ctx, n_max: int) -> None:
    _check(ctx, _lib.pa_reserve(ctx, n_max))


def pa_workspace_bytes(n: int) -> int:
    return int(_lib.pa_workspace_bytes(n))


def pa_transform_length(n: int) -> int:
    return int(_lib.pa_transform_length(n))


def _plan_dict(p) -> dict:
    return {"tile_log": p.tile_log, "strided_tile_log": p.strided_tile_log,
            "rows3_log": p.rows3_log, "passes": p.passes, "ms": float(p.ms)}


def pa_plan_candidates(n: int, max_count: int = 64) -> list[dict]:
    """Valid distinct transform geometries for blocks of n bits (default first)."""
    arr = (_Plan * max_count)()
    k = int(_lib.pa_plan_candidates(n, arr, max_count))
    return [_plan_dict(arr[i]) for i in range(k)]


def pa_plan_get(ctx, n: int) -> dict:
    p = _Plan()
    _check(ctx, _lib.pa_plan_get(ctx, n, ctypes.byref(p)))
    return _plan_dict(p)


def pa_plan_set(ctx, n: int, plan: dict | None) -> None:
    """Use this geometry for n's transform length (None: the default)."""
    if plan is None:
        _check(ctx, _lib.pa_plan_set(ctx, n, None))
        return
    p = _Plan(plan["tile_log"], plan.get("strided_tile_log", 0), plan.get("rows3_log", 0), 0, 0.0)
    _check(ctx, _lib.pa_plan_set(ctx, n, ctypes.byref(p)))


def pa_tune(ctx, n: int, reps: int = 3) -> dict:
    """Time every candidate geometry for n's length on the device; keep the fastest."""
    p = _Plan()
    _check(ctx, _lib.pa_tune(ctx, n, reps, ctypes.byref(p)))
    return _plan_dict(p)


def pa_toeplitz(ctx, key, t, seed_t: int, n: int, m: int) -> np.ndarray:
    """Toeplitz hash y = T x from host memory; t (n + m - 1 bits) or None: seeded."""
    key = _host_words(key, words(n), "key")
    tp = None
    if t is not None:
        t = _host_words(t, words(n + m - 1), "t")
        tp = t.ctypes.data_as(_u64p)
    out = np.zeros(max(words(m), 1), dtype=np.uint64)
    _check(ctx, _lib.pa_toeplitz(ctx, key.ctypes.data_as(_u64p), tp, seed_t & MASK64, n, m,
                                 out.ctypes.data_as(_u64p)))
    return out


def pa_toeplitz_async(ctx, d_key, d_t, seed_t: int, n: int, m: int, d_out, stream=None) -> None:
    """Queue the Toeplitz hash of device tensor d_key into d_out (d_t None: seeded)."""
    tptr = None if d_t is None else _dev_ptr(d_t, words(n + m - 1), "d_t")
    _check(ctx, _lib.pa_toeplitz_async(ctx, _dev_ptr(d_key, words(n), "d_key"), tptr,
                                       seed_t & MASK64, n, m, _dev_ptr(d_out, words(m), "d_out"),
                                       _stream_handle(stream)))


def pa_toeplitz_length(n: int, m: int) -> tuple[int, int]:
    """(transform length per piece, number of key pieces); (0, 0) when out of range."""
    pieces = _u64(0)
    L = int(_lib.pa_toeplitz_length(n, m, ctypes.byref(pieces)))
    return L, int(pieces.value)


def _job_array(jobs):
    """jobs: dicts with key/out device tensors, n, m, seed_a, seed_b and
    optional c/d device tensors."""
    arr = (_Job * len(jobs))()
    for i, j in enumerate(jobs):
        n, m = int(j["n"]), int(j["m"])
        arr[i].key = _dev_ptr(j["key"], words(n), "key")
        arr[i].out = _dev_ptr(j["out"], words(m), "out")
        arr[i].c = _dev_ptr(j["c"], words(n), "c") if j.get("c") is not None else None
        arr[i].d = _dev_ptr(j["d"], words(n), "d") if j.get("d") is not None else None
        arr[i].seed_a = int(j.get("seed_a", 0)) & MASK64
        arr[i].seed_b = int(j.get("seed_b", 0)) & MASK64
        arr[i].n, arr[i].m = n, m
        arr[i].status = -1
    return arr


def pa_hash_many(ctx, jobs, stream=None) -> list[int]:
    """Hash every block of `jobs` (see _job_array) and wait; per-block status."""
    arr = _job_array(jobs)
    _check(ctx, _lib.pa_hash_many(ctx, arr, len(jobs), _stream_handle(stream)))
    return [arr[i].status for i in range(len(jobs))]


class Batch:
    """pa_batch: a planned batch whose launches can be replayed (and captured
    into a HIP graph).  Keeps the job array alive with the batch.  mode:
    PA_BATCH_GROUPED (one launch per pass per length group) or
    PA_BATCH_PERSISTENT (one queue kernel; refused until validated on a GPU)."""

    def __init__(self, ctx, jobs, mode: int = PA_BATCH_GROUPED, wait_us: int = 0,
                 force_abort: bool = False):
        self.ctx = ctx
        self._jobs = _job_array(jobs)
        self._refs = jobs
        opts = _BatchOpts(int(mode), int(wait_us), int(bool(force_abort)))
        h = ctypes.c_void_p()
        _check(ctx, _lib.pa_batch_create_ex(ctx, self._jobs, len(jobs), ctypes.byref(opts),
                                            ctypes.byref(h)))
        self.h = h

    def result(self) -> int:
        """After the run's stream completed: PA_OK or PA_EDEVICE (a persistent
        dependency wait gave up)."""
        return int(_lib.pa_batch_result(self.h))

    @property
    def status(self) -> list[int]:
        return [self._jobs[i].status for i in range(len(self._jobs))]

    def run(self, stream=None):
        _check(self.ctx, _lib.pa_batch_run(self.h, _stream_handle(stream)))

    def capture(self, stream=None):
        _check(self.ctx, _lib.pa_batch_capture(self.h, _stream_handle(stream)))

    def tune(self, reps: int = 3):
        """Time every candidate geometry per length group and keep the fastest
        (drops a captured graph: capture again afterwards)."""
        _check(self.ctx, _lib.pa_batch_tune(self.h, int(reps)))

    def groups(self) -> list[dict]:
        """Per length group: transform length, block count and geometry."""
        out = []
        for i in range(int(_lib.pa_batch_groups(self.h))):
            L, cnt, p = ctypes.c_uint64(), ctypes.c_uint32(), _Plan()
            _check(self.ctx, _lib.pa_batch_group(self.h, i, ctypes.byref(L), ctypes.byref(cnt),
                                                 ctypes.byref(p)))
            out.append({"length": L.value, "blocks": cnt.value} | _plan_dict(p))
        return out

    def bytes(self) -> int:
        return int(_lib.pa_batch_bytes(self.h))

    def size(self) -> int:
        return int(_lib.pa_batch_size(self.h))

    def launches(self) -> int:
        return int(_lib.pa_batch_launches(self.h))

    def close(self):
        if self.h:
            _lib.pa_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """pa_server: continuous hashing of a request stream on one GPU."""

    def __init__(self, hbm_budget: int, slots: int = 8, max_n: int = 10**8, device: int = 0):
        opts = _ServerOpts(int(hbm_budget), int(slots), int(max_n))
        h = ctypes.c_void_p()
        rc = _lib.pa_server_create(int(device), ctypes.byref(opts), ctypes.byref(h))
        if rc != PA_OK:
            raise PAError(rc, pa_strerror(rc))
        self.h = h
        self._keep = {}

    def submit(self, key, seed_a: int, seed_b: int, n: int, m: int, out, ready=None) -> int:
        """key/out: device tensors (PA_SUBMIT_DEVICE) or host numpy uint64 arrays.
        ready: for device tensors still being written by queued work, a
        torch.cuda.Event recorded after that work (kept until the request ends)."""
        t = ctypes.c_uint64()
        ev = None
        if getattr(key, "is_cuda", False):
            kp, op, flags = _dev_ptr(key, words(n), "key"), _dev_ptr(out, words(m), "out"), 1
            if ready is not None:
                ev = getattr(ready, "cuda_event", ready)
        else:
            if ready is not None:
                raise ValueError("ready events apply to device requests only")
            if not (isinstance(out, np.ndarray) and out.dtype == np.uint64
                    and out.flags.c_contiguous and out.size >= words(m)):
                raise ValueError("out: need a contiguous uint64 array of ceil(m/64) words")
            key = _host_words(key, words(n), "key")
            kp, op, flags = key.ctypes.data, out.ctypes.data, 0
        rc = _lib.pa_server_submit_after(self.h, kp, seed_a & MASK64, seed_b & MASK64, n, m, op,
                                         flags, ev, ctypes.byref(t))
        if rc != PA_OK:
            raise PAError(rc, pa_strerror(rc))
        self._keep[t.value] = (key, out, ready)
        return t.value

    def wait(self, ticket: int) -> tuple[int, float]:
        st, lat = ctypes.c_int(), ctypes.c_double()
        rc = _lib.pa_server_wait(self.h, ticket, ctypes.byref(st), ctypes.byref(lat))
        if rc != PA_OK:
            raise PAError(rc, pa_strerror(rc))
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def drain(self):
        _lib.pa_server_drain(self.h)
        self._keep.clear()

    def stats(self) -> dict:
        st = _ServerStats()
        _lib.pa_server_get_stats(self.h, ctypes.byref(st))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def run_trace(self, jobs, arrival_s, device: bool = True):
        """Open-loop replay: jobs[i] submitted at arrival_s[i] seconds; returns
        (latencies_ms, statuses).  device=True: dicts as for Batch (device
        tensors, complete before the call); device=False: key and out are host
        numpy uint64 arrays, so every latency includes the key's copy to the
        device and the result's copy back."""
        k = len(jobs)
        keep = []                       # host copies that must outlive the call
        if device:
            arr = _job_array(jobs)
        else:
            arr = (_Job * k)()
            for i, j in enumerate(jobs):
                n, m = int(j["n"]), int(j["m"])
                key = _host_words(j["key"], words(n), "key")
                keep.append(key)
                out = j["out"]
                if not (isinstance(out, np.ndarray) and out.dtype == np.uint64
                        and out.flags.c_contiguous and out.size >= words(m)):
                    raise ValueError("out: need a contiguous uint64 array of ceil(m/64) words")
                arr[i].key, arr[i].out = key.ctypes.data, out.ctypes.data
                arr[i].seed_a = int(j.get("seed_a", 0)) & MASK64
                arr[i].seed_b = int(j.get("seed_b", 0)) & MASK64
                arr[i].n, arr[i].m = n, m
        t = (ctypes.c_double * k)(*[float(x) for x in arrival_s])
        lat = (ctypes.c_double * k)()
        st = (ctypes.c_int * k)()
        rc = _lib.pa_server_run_trace(self.h, arr, t, k, PA_SUBMIT_DEVICE if device else 0, lat, st)
        if rc != PA_OK:
            raise PAError(rc, pa_strerror(rc))
        return list(lat), list(st)

    def close(self):
        if self.h:
            _lib.pa_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Owns one pa_ctx; a convenience wrapper over the functions above."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, tune_cache: str | None = None):
        self.ctx = pa_init(device, hbm_budget, tune_cache)

    def close(self):
        if self.ctx:
            pa_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hash(self, key, seed_a, seed_b, n, m):
        return pa_hash(self.ctx, key, seed_a, seed_b, n, m)

    def hash_ex(self, key, c, d, n, m):
        return pa_hash_ex(self.ctx, key, c, d, n, m)

    def hash_async(self, d_key, seed_a, seed_b, n, m, d_out, stream=None):
        pa_hash_async(self.ctx, d_key, seed_a, seed_b, n, m, d_out, stream)

    def profile(self, d_key, seed_a, seed_b, n, m, d_out, stream=None):
        return pa_hash_profile(self.ctx, d_key, seed_a, seed_b, n, m, d_out, stream)

    def reserve(self, n_max):
        pa_reserve(self.ctx, n_max)
