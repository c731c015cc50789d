"""CPU checks of the host tables behind the register-phase kernel: the C++
harness tests/host/check_fast_tables.cpp is compiled against the library's
table builder (host code only, no GPU) and run here."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_01903_amd", "csrc")


def test_register_kernel_tables():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "check")
        cmd = ["hipcc", "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
               os.path.join(ROOT, "tests", "host", "check_fast_tables.cpp"),
               os.path.join(CSRC, "fsi_tables.cpp"), "-o", exe]
        try:
            subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
        except FileNotFoundError:
            pytest.skip("hipcc not available")
        out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
        assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr
