"""CPU-side checks of the C ABI library: it loads, exports every function the
header declares, and its host-only helpers and argument checks behave."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (load torch's HIP runtime before libpa, as the binding does)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")
LIB = os.path.join(ROOT, "paper_1910_04429_amd", "libpa.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["pa_init", "pa_destroy", "pa_strerror", "pa_last_error", "pa_hash",
                 "pa_hash_ex", "pa_hash_async", "pa_hash_profile", "pa_reserve",
                 "pa_workspace_bytes", "pa_transform_length"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_helpers():
    import paper_1910_04429_amd as pa
    # L = smallest 2^k (k >= 6) or, from 2^18 on, 3 * 2^k with L >= 2D - 1, for
    # D = ceil(n / 64) digits over five primes or D = ceil(n / 96) over seven,
    # whichever needs less transform work
    assert pa.pa_transform_length(1) == 64
    assert pa.pa_transform_length(1_000_000) == 1 << 15        # 64-bit: 2D - 1 = 31249
    assert pa.pa_transform_length(10_000_000) == 1 << 18       # 96-bit: 208333
    assert pa.pa_transform_length(100_000_000) == 1 << 21      # 96-bit: 2083333
    assert pa.pa_transform_length(pa.PA_MAX_N) == 1 << 24      # 64-bit: 2^24 - 1
    assert pa.pa_transform_length(pa.PA_MAX_N + 1) == 0
    assert pa.pa_transform_length(0) == 0
    assert pa.pa_workspace_bytes(100_000_000) >= 2 * 7 * 4 * (1 << 21)
    assert pa.pa_strerror(pa.PA_EINVAL) == "invalid argument"
    assert pa.pa_strerror(pa.PA_EIO) == "tuning cache file error"


def test_noalloc_scratch_holds_every_block_up_to_3_2_25_bits():
    """The allocation-free entry point's scratch covers the spectra and carry
    state (plus at most 768 bytes of alignment) of every block of at most
    3 * 2^25 bits, the paper's largest block of 10^8 bits included."""
    import paper_1910_04429_amd as pa
    top = 3 << 25
    worst = max(pa.pa_workspace_bytes(n) for n in list(range(64, top, 6144)) + [10**8, top])
    assert worst + 768 <= pa.PA_NOALLOC_MAX_BYTES
    assert pa.pa_workspace_bytes(top + 1) + 768 > pa.PA_NOALLOC_MAX_BYTES


def test_null_context_is_rejected():
    lib = ctypes.CDLL(LIB)
    lib.pa_hash.restype = ctypes.c_int
    lib.pa_hash.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_uint64] * 4 + [ctypes.c_void_p]
    assert lib.pa_hash(None, None, 0, 0, 64, 8, None) == 1   # PA_EINVAL
    lib.pa_destroy.argtypes = [ctypes.c_void_p]
    lib.pa_destroy(None)


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1910_04429_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def test_init_without_gpu_fails_cleanly():
    import paper_1910_04429_amd as pa
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(pa.PAError) as e:
        pa.pa_init(0)
    assert e.value.status == pa.PA_ENODEV


def test_single_hip_runtime_in_process():
    """The binding must share torch's HIP runtime, not load a second one."""
    import paper_1910_04429_amd  # noqa: F401
    with open("/proc/self/maps") as f:
        paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(paths) == 1, paths


def test_build_scripts_load_before_the_libraries_exist():
    """build() must work on a fresh checkout: its build scripts load by file
    path, without importing the packages (which refuse to load before their
    libraries exist)."""
    import subprocess
    import sys
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")
    code = ("import sys, __graft_entry__ as g, os; "
            "g._load_script(os.path.join(g.ROOT, 'paper_1910_04429_amd', 'build.py'), 'a'); "
            "g._load_script(os.path.join(g.ROOT, 'oracle', 'build.py'), 'b'); "
            "assert 'paper_1910_04429_amd' not in sys.modules and 'oracle' not in sys.modules")
    subprocess.run([sys.executable, "-c", code], cwd=root, check=True)
