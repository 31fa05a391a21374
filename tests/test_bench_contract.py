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


def test_oracle_sample_takes_whole_chunks_until_the_target_or_the_time():
    calls = []
    starts = [0, 3, 6, 9, 10]
    comps = lambda r0, r1: sum(10 - i for i in range(r0, r1))
    r0, r1, done, dt = bench.oracle_sample(lambda a, b: calls.append((a, b)), comps, starts,
                                           1e18, 0.0)
    assert calls == [(0, 3)] and (r0, r1) == (0, 3) and done == 10 + 9 + 8  # at least one chunk
    calls.clear()
    r0, r1, done, dt = bench.oracle_sample(lambda a, b: calls.append((a, b)), comps, starts,
                                           1e18, 1e9)
    assert calls == [(0, 3), (3, 6), (6, 9), (9, 10)] and r1 == 10 and done == 55
    calls.clear()  # stops once the comparison target is reached
    r0, r1, done, dt = bench.oracle_sample(lambda a, b: calls.append((a, b)), comps, starts,
                                           30, 1e9)
    assert calls == [(0, 3), (3, 6)] and done == 27 + 18
    calls.clear()  # ranges that start past row 0 (the one-thread 3-way sample)
    r0, r1, done, dt = bench.oracle_sample(lambda a, b: calls.append((a, b)), comps, [7, 9, 10],
                                           1e18, 1e9)
    assert calls == [(7, 9), (9, 10)] and (r0, r1) == (7, 10) and done == 3 + 2 + 1


def test_cpu_baseline_reports_model_threads_one_core_and_extrapolation():
    import argparse
    import time
    args = argparse.Namespace(cpu_comparisons=50, cpu_seconds=1e9, cpu_one_core_seconds=1e9)

    def call(a, b):
        time.sleep(0.001 * (b - a))

    out = bench.cpu_baseline(args, call, lambda a, b: 10 * (b - a), 20, 200, "rows", chunk=2)
    assert out["kind"] == "oracle" and out["unit"] == "comparisons/s"
    assert out["threads"] == out["cores"] >= 1 and out["cpu_model"]
    assert out["sample_comparisons"] == 60  # whole chunks until >= 50
    assert abs(out["extrapolated_full_s"] - 200 / out["value"]) < 1e-9
    assert "shortfall" not in out
    assert out["single_core"]["value"] > 0 and "1 thread" in out["single_core"]["sample"]


def test_operand_format_and_peak_follow_the_library():
    fmt, peak, dt = bench.mfma_format(65536)
    assert (fmt, peak, dt) == ("fp4", bench.FP4_PEAK_TFLOPS, "fp4")
    fmt, peak, dt = bench.mfma_format((1 << 22) + 1)
    assert (fmt, peak, dt) == ("int8", bench.INT8_PEAK_TOPS, "i8")
    assert bench.mfma_format(65536, "int8") == ("int8", bench.INT8_PEAK_TOPS, "i8")
    assert bench.mfma_format(1000, "fp4") == ("fp4", bench.FP4_PEAK_TFLOPS, "fp4")


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
