"""Host check of the MFMA kernels' A tables and lane-to-line maps (paper_2003_12787_amd/csrc/mfma_tables.cpp),
built with g++ (no GPU): a double-precision emulation of the products with the kernels' operand layouts must
give the documented sums of piece products exactly, and the order 8-9 line maps must cover every line once
per role, conflict-free in the LDS banks at n = 10 (tests/host/mfma_tables_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2003_12787_amd", "csrc")


def test_mfma_tables_emulated(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tables")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", CSRC, "-o", exe, os.path.join(CSRC, "mfma_tables.cpp"),
                           os.path.join(HERE, "host", "mfma_tables_driver.cpp")])
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failures" in out, out[-4000:]
    assert "n=10: worst bank multiplicity per wave: owner 1, y-role 1, z-role 1" in out, out
