"""Host-side test of the MD graph cache's key and eviction logic: a plain
C++ program built from the library's graph_cache.h with g++ (no GPU)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_graph_cache_key_and_eviction(tmp_path):
    exe = str(tmp_path / "graph_cache_check")
    src = os.path.join(ROOT, "tests", "graph_cache_check.cpp")
    inc = os.path.join(ROOT, "paper_2502_06073_amd", "csrc")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", inc, src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "eviction ok" in r.stdout
