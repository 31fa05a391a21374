"""The library's host code (argument validation of every entry point, the
batched entry point's tune-table parse, descriptors, largest-first work list
and cache key, the timing hooks) under AddressSanitizer + UndefinedBehavior-
Sanitizer, without a GPU: the HIP sources are compiled with the sanitizers on
their host side only, linked with tests/native/abi_sanitize.cpp, and run."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1705_08213_amd", "csrc")

def _sources():
    from paper_1705_08213_amd.build import SOURCES
    return [os.path.splitext(f)[0] for f in SOURCES]


SOURCES = _sources()
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def test_library_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    common = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN,
              "-I", os.path.join(ROOT, "include")]

    def compile_one(name):
        src = (os.path.join(CSRC, name + ".hip") if name != "driver"
               else os.path.join(HERE, "native", "abi_sanitize.cpp"))
        obj = str(tmp_path / (name + ".o"))
        r = subprocess.run([*common, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES + ["driver"]))
    exe = str(tmp_path / "abi_sanitize")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", *SAN, *objs, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, (out.stdout + out.stderr)[-3000:]
    assert out.stdout.startswith("ok "), out.stdout + out.stderr
    assert "ERROR: AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr
