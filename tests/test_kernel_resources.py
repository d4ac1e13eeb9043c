"""Compile-time guard (CPU): no kernel of libpa may use scratch memory or spill
VGPRs.  Private-memory traffic in a pass kernel is a silent several-fold
slowdown, so it is caught here rather than on the GPU."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_04429_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


@pytest.mark.skipif(HIPCC is None, reason="hipcc not available")
@pytest.mark.parametrize("src", ["ntt.hip", "carry.hip", "toeplitz.hip"])
def test_no_scratch_no_vgpr_spill(src, tmp_path):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
           "--cuda-device-only", "-c", os.path.join(CSRC, src), "-o", str(tmp_path / "k.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    names = re.findall(r"Function Name: (\S+)", out)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out)]
    spills = [int(x) for x in re.findall(r"VGPRs Spill: (\d+)", out)]
    assert names and len(scratch) == len(names) == len(spills)
    for n, s, v in zip(names, scratch, spills):
        assert s == 0, f"{n} uses {s} bytes/lane of scratch"
        assert v == 0, f"{n} spills {v} VGPRs"
