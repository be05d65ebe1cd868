"""Host-side test of the edge-tile tuner's result cache: a plain C++ program
built from the library's tune_cache.h with g++ (no GPU)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tune_cache_round_trip_and_update(tmp_path):
    exe = str(tmp_path / "tune_cache_check")
    src = os.path.join(ROOT, "tests", "tune_cache_check.cpp")
    inc = os.path.join(ROOT, "paper_2502_06073_amd", "csrc")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", inc, src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe, str(tmp_path / "tune.json")], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "tune cache ok" in r.stdout
