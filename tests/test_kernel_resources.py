"""Compile-time guards (CPU) on the kernels' registers.

No kernel of libpa may use scratch memory or spill VGPRs: private-memory
traffic in a pass kernel is a silent several-fold slowdown.  Scalar registers
that do not fit are kept in VGPR lanes (v_writelane / v_readlane, VALU
instructions).  In the pass kernels that traffic must stay out of the
innermost loops that do the arithmetic (the per-DFT loops, at least 64 VALU
instructions per iteration) but for a stray reload or two that the register
allocator places at a loop latch: at most 2 lane instructions per such loop
and at most 1.5% of its VALU instructions.  (A kernel whose scalar registers
are squeezed, as the one for all kinds of pass was, or one forced to eight
waves per SIMD, has tens to hundreds of them per loop.)  The short load/store
sweeps may reload a bound.  Caught here rather than on the GPU.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_04429_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


def innermost_loops(asm_lines):
    """(first, last) line of each loop that contains no other loop: a backward
    branch to a label, taken as a loop from the label to the branch."""
    labels = {}
    for i, line in enumerate(asm_lines):
        m = re.match(r"^(\.LBB\d+_\d+):", line)
        if m:
            labels[m.group(1)] = i
    loops = []
    for i, line in enumerate(asm_lines):
        m = re.search(r"s_(?:cbranch_\w+|branch)\s+(\.LBB\d+_\d+)", line)
        if m and m.group(1) in labels and labels[m.group(1)] < i:
            loops.append((labels[m.group(1)], i))
    return [a for a in loops
            if not any(b != a and a[0] <= b[0] and b[1] <= a[1] for b in loops)]


def kernels_of(asm):
    """Kernel name -> its lines, from a device assembly file."""
    out, cur = {}, None
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            cur = m.group(1)
            out[cur] = []
        elif cur:
            out[cur].append(line)
            if "s_endpgm" in line:
                cur = None
    return out


@pytest.mark.skipif(HIPCC is None, reason="hipcc not available")
@pytest.mark.parametrize("src", ["ntt.hip", "carry.hip", "toeplitz.hip"])
def test_no_scratch_no_vgpr_spill(src, tmp_path):
    asm_path = tmp_path / "k.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", str(asm_path),
           "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    names = re.findall(r"Function Name: (\S+)", out)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out)]
    spills = [int(x) for x in re.findall(r"VGPRs Spill: (\d+)", out)]
    assert names and len(scratch) == len(names) == len(spills)
    for n, s, v in zip(names, scratch, spills):
        assert s == 0, f"{n} uses {s} bytes/lane of scratch"
        assert v == 0, f"{n} spills {v} VGPRs"
    if src != "ntt.hip":
        return
    kernels = kernels_of(asm_path.read_text())
    passes = [k for k in kernels if "k_pass" in k]
    assert len(passes) == 18            # two layouts x (four kinds x single/batch + one-pass fused)
    for k in passes:
        lines = kernels[k]
        loops = innermost_loops(lines)
        assert loops, k
        heavy = 0
        for a, b in loops:
            body = lines[a:b + 1]
            valu = sum(1 for x in body if x.startswith("\tv_"))
            if valu < 64:
                continue
            heavy += 1
            lane = [x for x in body if "v_readlane_b32" in x or "v_writelane_b32" in x]
            assert len(lane) <= 2 and len(lane) <= 0.015 * valu, \
                f"{k}: scalar-register spill traffic inside an arithmetic loop: {lane}"
        assert heavy, k
