"""The work enumerations of the library, compiled for the host from its own
header and checked by brute force: the 3-way work units (tile-pair major, XCD
remap) cover every staged triple exactly once, and the 2-way strip order of
squares maps one to one onto each row range's squares."""
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
