"""bench.py's host-side contract, without a GPU: the multi-GPU refusal, the
bounded oracle baseline, the operand format and peak it reports, and the
traffic figure it takes from a committed profile only while the kernel
sources hash to the profiled ones."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_oracle_sample_takes_whole_chunks_until_the_time_is_spent():
    calls = []
    rows, units, dt = bench.oracle_sample(lambda r0, r1: calls.append((r0, r1)),
                                          lambda i: 10 - i, 10, 3, 0.0)
    assert calls == [(0, 3)] and rows == 3 and units == 10 + 9 + 8  # at least one chunk
    calls.clear()
    rows, units, dt = bench.oracle_sample(lambda r0, r1: calls.append((r0, r1)),
                                          lambda i: 1, 10, 3, 1e9)
    assert calls == [(0, 3), (3, 6), (6, 9), (9, 10)] and rows == 10 and units == 10


def test_operand_format_and_peak_follow_the_library():
    fmt, peak, dt = bench.mfma_format(65536)
    assert (fmt, peak, dt) == ("fp4", bench.FP4_PEAK_TFLOPS, "fp4")
    fmt, peak, dt = bench.mfma_format((1 << 22) + 1)
    assert (fmt, peak, dt) == ("int8", bench.INT8_PEAK_TOPS, "i8")


def test_committed_traffic_needs_the_profiled_sources(tmp_path):
    # a summary written for the current sources gives its figure; one for any
    # other source set (or stale, or absent) gives none
    import hashlib
    h = hashlib.sha256(b"".join(open(os.path.join(bench.ROOT, f), "rb").read()
                                for f in bench.MFMA2_SOURCES)).hexdigest()[:16]
    prof = tmp_path / "summary.md"
    prof.write_text(f"traffic_bytes_per_launch: 123456789\nkernel_source_sha256_16: {h}\n")
    assert bench.committed_traffic(bench.MFMA2_SOURCES, str(prof)) == 123456789
    assert bench.committed_traffic(bench.MFMA3_SOURCES, str(prof)) is None
    prof.write_text("traffic_bytes_per_launch: 123456789\nkernel_source_sha256_16: 0123456789abcdef\n")
    assert bench.committed_traffic(bench.MFMA2_SOURCES, str(prof)) is None
    assert bench.committed_traffic(bench.MFMA2_SOURCES, str(tmp_path / "absent.md")) is None
