"""The library's host code (layout, CG tables, stage costs, workspace plan)
under AddressSanitizer: its C++ sources are compiled with host-side ASan
(device code untouched), linked with the built HIP objects and a driver that
sweeps l_max 0-3, 1-3 layers, 8-128 channels, both mixings and four widths
(no GPU call is made)."""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_06073_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2502_06073_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_host_entry_points_under_asan(tmp_path):
    hip_objs = sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
    if not hip_objs:
        pytest.skip("library not built (python -m paper_2502_06073_amd.build)")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    fl = ["-O1", "-g", "-fPIC", "-std=c++20", "--offload-arch=gfx950", "-Wno-unused-command-line-argument"]
    asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("model", "weights", "api", "trace", "tuner"):
        o = str(tmp_path / f"{src}.o")
        r = subprocess.run([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, f"{src}.cpp"), "-o", o] + inc + fl + asan,
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(o)
    drv = str(tmp_path / "driver.o")
    r = subprocess.run([HIPCC, "-c", os.path.join(ROOT, "tests", "host_abi_sweep.cpp"), "-o", drv, "-O1", "-g",
                        "-std=c++20"] + inc + asan, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "sweep")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-o", exe, drv] + objs + hip_objs + asan,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ok " in r.stdout and "AddressSanitizer" not in r.stderr
