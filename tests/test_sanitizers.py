"""The oracle and the library's host-side cache parser under AddressSanitizer + UndefinedBehaviorSanitizer
(and the oracle's worker threads under ThreadSanitizer), built with gcc/g++ on the CPU.

The drivers in tests/sanitize/ call every oracle entry point on small random inputs of every physics, and the
cache parser on valid, round-tripped, truncated and malformed texts. A run passes when the driver's own checks
hold and the sanitizers report nothing (the builds abort on the first report)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _build_and_run(tmp_path, compiler, sources, flags, extra_env=None):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / "driver")
    subprocess.check_call([compiler, *flags, "-o", exe, *sources, "-lm", "-lpthread"])
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env.update(extra_env or {})
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for marker in ("runtime error", "AddressSanitizer", "LeakSanitizer", "ThreadSanitizer"):
        assert marker not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [os.path.join(ROOT, "oracle", "stp_oracle.c"),
                                           os.path.join(HERE, "sanitize", "oracle_driver.c")],
                         ["-std=c11", *SAN], {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1"})
    assert "0 failures" in out


def test_oracle_threads_under_tsan(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [os.path.join(ROOT, "oracle", "stp_oracle.c"),
                                           os.path.join(HERE, "sanitize", "oracle_driver.c")],
                         ["-std=c11", "-g", "-O1", "-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert "0 failures" in out


def test_tune_cache_parser_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2003_12787_amd", "csrc")
    out = _build_and_run(tmp_path, "g++", [os.path.join(csrc, "tune_cache.cpp"),
                                           os.path.join(HERE, "sanitize", "cache_driver.cpp")],
                         ["-std=c++17", "-I", csrc, *SAN], {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1"})
    assert "0 failures" in out
