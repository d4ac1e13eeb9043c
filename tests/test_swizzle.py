"""Host check of the pass kernels' LDS tile layout (swizzle.h): built with the
host compiler and run on the CPU.  A map that left a tile would make a step
address LDS outside it, so the properties are checked exhaustively for every
tile size here rather than found on the GPU."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1910_04429_amd", "csrc")


def test_tile_swizzle_properties(tmp_path):
    exe = tmp_path / "swizzle_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", CSRC,
                    os.path.join(HERE, "native", "swizzle_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("ok")
