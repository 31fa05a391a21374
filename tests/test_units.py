"""The 3-way work-unit enumeration of the library (tile-pair major, XCD
remap), compiled for the host from the library's own header and checked by
brute force: every staged triple is covered by exactly one unit."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_unit_enumeration_covers_each_triple_once(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "units_check"
    r = subprocess.run([hipcc, "-O1", "-std=c++17", os.path.join(HERE, "native", "units_check.cpp"),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
