"""Host check of the carry-transfer function algebra (carryfn.h) used by the
carry kernels: built with the host compiler and run on the CPU.

Random GPU parity inputs almost never produce a column sum within 3 of a
2^32 boundary (the only case where a position's function has a step inside
0..3), so the algebra is checked exhaustively here instead."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1910_04429_amd", "csrc")


def test_carry_function_algebra(tmp_path):
    exe = tmp_path / "carryfn_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", CSRC,
                    os.path.join(HERE, "native", "carryfn_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("ok")
