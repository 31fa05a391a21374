#!/usr/bin/env python3
"""Throughput of the CCC tally hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2] [--operands auto]

A step is one call of the library's entry point for the workload (1-way
count pass, tally kernel and fused FP64 epilogue writing every table and CCC
value) on inputs already resident in HBM.  The default workload is the large
2-way configuration (n_v = 32768 vectors x n_f = 65536 fields, per-vector
allele frequency ~ Beta(1/2,1/2), Hardy-Weinberg genotypes, 1% missing) on
the MFMA path with the default operands (fp4 at this size); the same call
with int8 operands (the modified-GEMM tally on the int8 matrix cores) and
the popcount path are timed on the same input beside it.  The CPU oracle is
timed on a bounded sample of the same input.  Prints one JSON line.

Other workloads (--config): c1 (2-way 512 x 1000, popcount path), c2c (the
c2 shape with no missing entries: the complete-data path), c3 (3-way
2048 x 16384), c3c (the c3 shape with no missing entries), c4 (64 batched
2-way problems), c5 (2-way off-diagonal block 16384 x 16384 over 131072
fields in 8 chunks), c2m (multi-allelic 2-way, 16384 x 32768, 4 states).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 MFMA, 5.0 POP/s
FP4_PEAK_TFLOPS = 10100.0    # MI355X dense fp4 (e2m1) MFMA, 10.1 PFLOP/s


def mfma_format(n_f, operands="auto"):
    """(operand format, dense peak in T(FL)OP/s, dtype tag) of the MFMA kernels
    over n_f fields: the forced format, else the one the library picks."""
    import paper_1705_08213_amd as ccc
    fmt = operands if operands != "auto" else ccc.mfma_operands(n_f)
    return (fmt, FP4_PEAK_TFLOPS, "fp4") if fmt == "fp4" else (fmt, INT8_PEAK_TOPS, "i8")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def committed_traffic(kernel_sources, profile):
    """HBM bytes per launch recorded in a committed rocprofv3 summary, or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    import re
    try:
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                    for f in kernel_sources)).hexdigest()[:16]
        text = open(os.path.join(ROOT, profile)).read()
    except OSError:
        return None
    m1 = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    m2 = re.search(r"kernel_source_sha256_16: ([0-9a-f]+)", text)
    if m1 and m2 and m2.group(1) == h:
        return int(m1.group(1))
    return None


MFMA2_SOURCES = ["paper_1705_08213_amd/csrc/mfma2.hip", "paper_1705_08213_amd/csrc/tile2.h",
                 "paper_1705_08213_amd/csrc/common.h", "paper_1705_08213_amd/csrc/kernels.h"]
MULTI2_SOURCES = ["paper_1705_08213_amd/csrc/multi2.hip", "paper_1705_08213_amd/csrc/tile2.h",
                  "paper_1705_08213_amd/csrc/common.h", "paper_1705_08213_amd/csrc/kernels.h"]
MFMA3_SOURCES = ["paper_1705_08213_amd/csrc/mfma3.hip", "paper_1705_08213_amd/csrc/tile3.h",
                 "paper_1705_08213_amd/csrc/tile2.h", "paper_1705_08213_amd/csrc/common.h",
                 "paper_1705_08213_amd/csrc/kernels.h"]


def timing_query(lib, name):
    cnt = ctypes.c_int(0)
    lib.ccc_timing_query.restype = ctypes.c_double
    lib.ccc_timing_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
    ms = lib.ccc_timing_query(name.encode(), ctypes.byref(cnt))
    return ms, cnt.value


def timed(fn, steps, warmup, lib, kernel):
    """Run fn warmup+steps times; returns (ms per step, mean kernel ms, launches)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    lib.ccc_timing_reset()
    lib.ccc_timing_enable(1)
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    lib.ccc_timing_enable(0)
    total = e0.elapsed_time(e1)
    kms, kn = timing_query(lib, kernel)
    lib.ccc_timing_reset()
    return total / steps, (kms / kn if kn else None), kn


def oracle_sample(call, comps_of, starts, target, seconds):
    """Runs call(r0, r1) over the consecutive row ranges starting at `starts`
    until `target` comparisons are done or `seconds` of time have passed (at
    least one range); returns (first row, end row, comparisons, s)."""
    done, dt = 0, 0.0
    r0 = starts[0]
    r = r0
    for r1 in starts[1:]:
        if r > r0 and (done >= target or dt >= seconds):
            break
        t = time.perf_counter()
        call(r, r1)
        dt += time.perf_counter() - t
        done += comps_of(r, r1)
        r = r1
    return r0, r, done, dt


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, call, comps_of, n_rows, total, what, chunk=8, one_core_rows=None):
    """The CPU oracle (plain loops, OpenMP over the inner index) on the same
    input: with every host thread over consecutive row chunks from row 0 until
    --cpu-comparisons comparisons are done or --cpu-seconds have passed, then
    on one thread over `one_core_rows` (default: row chunks from row 0) for
    --cpu-one-core-seconds.  `comps_of(r0, r1)` counts the comparisons of rows
    [r0, r1); `total` is the whole workload's count, for the extrapolated
    full-run time."""
    import oracle
    threads = oracle.num_threads()
    log(f"timing the CPU oracle on {threads} threads (up to {args.cpu_seconds:g} s)")
    starts = list(range(0, n_rows, chunk)) + [n_rows]
    r0, r1, done, dt = oracle_sample(call, comps_of, starts, args.cpu_comparisons,
                                     args.cpu_seconds)
    out = dict(value=done / dt, unit="comparisons/s", cores=threads, kind="oracle",
               sample=f"{what} with first index in [{r0},{r1}) of the same input "
                      f"({done:.3e} comparisons, {dt:.1f} s on {threads} threads)",
               cpu_model=cpu_model(), threads=threads, sample_comparisons=done,
               sample_seconds=dt, extrapolated_full_s=total / (done / dt))
    if done < args.cpu_comparisons:
        out["shortfall"] = (f"sample stopped at {args.cpu_seconds:g} s, below the "
                            f"{args.cpu_comparisons:.0e}-comparison target")
    if args.cpu_one_core_seconds > 0:
        log(f"timing the CPU oracle on 1 thread (up to {args.cpu_one_core_seconds:g} s)")
        starts1 = one_core_rows if one_core_rows is not None else list(range(0, n_rows, 1)) + [n_rows]
        oracle.set_num_threads(1)
        try:
            a0, a1, done1, dt1 = oracle_sample(call, comps_of, starts1, float("inf"),
                                               args.cpu_one_core_seconds)
        finally:
            oracle.set_num_threads(threads)
        out["single_core"] = dict(value=done1 / dt1, unit="comparisons/s",
                                  sample=f"{what} with first index in [{a0},{a1}) "
                                         f"({done1:.3e} comparisons, {dt1:.1f} s on 1 thread)",
                                  extrapolated_full_s=total / (done1 / dt1))
    return out


def cpu_baseline_2way(args, v, n_f):
    """The oracle on rows [0, r) x all later vectors."""
    import oracle
    n_v = v.shape[0]
    pairs = lambda r0, r1: sum(n_v - 1 - i for i in range(r0, r1))
    return cpu_baseline(args, lambda r0, r1: oracle.two_way(v, n_f, r0, r1, with_ccc=True),
                        lambda r0, r1: pairs(r0, r1) * n_f, n_v, n_v * (n_v - 1) // 2 * n_f,
                        "pairs (i, j > i)")


def cpu_baseline_3way(args, v, n_f):
    """The oracle on the triples whose first index is in a row range: from row
    0 on all threads, and from the end (rows with few triples) on one."""
    import oracle
    n_v = v.shape[0]
    tri = lambda r0, r1: sum((n_v - 1 - i) * (n_v - 2 - i) // 2 for i in range(r0, r1))
    # one thread: the last rows, in ranges of about 2e8 comparisons each
    tail, r, acc = [n_v - 2], n_v - 2, 0
    while r > 0 and len(tail) < 64:
        r -= 1
        acc += (n_v - 1 - r) * (n_v - 2 - r) // 2 * n_f
        if acc >= 2e8:
            tail.append(r)
            acc = 0
    tail = tail[::-1]
    return cpu_baseline(args, lambda r0, r1: oracle.three_way(v, n_f, r0, r1, with_ccc=True),
                        lambda r0, r1: tri(r0, r1) * n_f, n_v, tri(0, n_v) * n_f,
                        "triples (i, j > i, k > j)", chunk=1, one_core_rows=tail)


def bench_2way(args, lib, n_v, n_f, missing, gen, path, workload):
    import torch
    import paper_1705_08213_amd as ccc
    import synth
    log(f"generating {n_v} x {n_f} input")
    v = (synth.beta_hw if gen == "beta_hw" else synth.uniform)(n_v, n_f, seed=0,
                                                                missing=missing)
    dv = torch.from_numpy(v).cuda()
    P = ccc.n_pairs(n_v)
    tables = torch.empty((P, 4), dtype=torch.int32, device="cuda")
    cc = torch.empty((P, 4), dtype=torch.float64, device="cuda")
    counts = torch.empty((n_v, 4), dtype=torch.int32, device="cuda")
    kernel = "mfma2" if path == "mfma" else "pop2"

    def step(p=path, operands=args.operands if path == "mfma" else "auto"):
        ccc.ccc_2way(dv, n_f, tables, cc, counts, path=p, operands=operands)

    log(f"timing {path}: {args.warmup} warmup + {args.steps} steps")
    ms, kms, _ = timed(step, args.steps, args.warmup, lib, kernel)
    comps = P * n_f
    rate = comps / (ms / 1e3)
    out = dict(metric="CCC comparisons/sec (pairs*n_f), bit-exact tables", value=rate,
               unit="comparisons/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype=mfma_format(n_f)[2] if path == "mfma" else "u32", data="synthetic",
               config=dict(workload=workload, n_v=n_v, n_f=n_f, missing=missing, path=path))
    if path == "mfma":
        # 4 MACs per comparison (four operand-plane products); with no missing
        # entry anywhere every tile takes the one-plane complete-data form (1 MAC)
        fmt, peak, _ = mfma_format(n_f, args.operands)
        out["config"]["operands"] = fmt
        ops = (2.0 if missing == 0.0 else 8.0) * comps
        ach = ops / (kms / 1e3) / 1e12
        traffic = None
        if (n_v, n_f) == (32768, 65536) and fmt == "fp4":
            traffic = committed_traffic(
                MFMA2_SOURCES, "profiles/mfma2_2way_n32768_f65536_traffic.md" if missing > 0.0
                else "profiles/mfma2_2way_complete_n32768_f65536.md")
        out["roofline"] = dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                               frac=ach / peak, traffic=traffic,
                               traffic_unit="bytes per launch (FETCH_SIZE+WRITE_SIZE, scaled)",
                               algorithmic_bytes=n_v * ((n_f + 3) // 4) + 48 * P + 32 * n_v,
                               # every row complete: the complete-data kernel does the
                               # work (the general one exits at once); kernel_ms is the
                               # HIP-event interval around the launcher's kernels
                               kernel="mfma2_complete_kernel" if missing == 0.0
                               else "mfma2_kernel", kernel_ms=kms, operands=fmt,
                               ops_per_comparison=2 if missing == 0.0 else 8)
        other = {"fp4": "int8", "int8": "fp4"}[fmt]
        if args.other_steps > 0 and mfma_format(n_f, other)[0] == other and (
                other == "int8" or n_f <= (1 << 22)):
            # the same call with the other operand format: int8 is the paper's
            # modified-GEMM tally on the int8 matrix cores
            log(f"timing mfma with {other} operands: 1 warmup + {args.other_steps} steps")
            oms, okms, _ = timed(lambda: step("mfma", other), args.other_steps, 1, lib, "mfma2")
            opeak = mfma_format(n_f, other)[1]
            oach = ops / (okms / 1e3) / 1e12
            out["mfma_" + other] = dict(value=comps / (oms / 1e3), ms_per_step=oms,
                                        kernel_ms=okms, achieved=oach, peak=opeak,
                                        unit="TFLOP/s" if other == "fp4" else "TOP/s",
                                        frac=oach / opeak)
        if args.select_threshold is not None:
            thr = args.select_threshold
            log(f"timing threshold selection at {thr}")
            found = {}

            def sel_step():
                found["n"] = ccc.ccc_2way_select(dv, n_f, thr, cap=1 << 22, counts=counts)[0]

            sms, _, _ = timed(sel_step, args.steps, 1, lib, "mfma2")
            out["select"] = dict(threshold=thr, kept=found["n"], ms_per_step=sms,
                                 value=comps / (sms / 1e3),
                                 note="ccc_2way_select: only pairs with a CCC value >= "
                                      "threshold are written (includes a count read-back)")
        if args.pop_steps > 0:
            log(f"timing popcount: 1 warmup + {args.pop_steps} steps")
            pms, pkms, _ = timed(lambda: step("popcount"), args.pop_steps, 1, lib, "pop2")
            prate = comps / (pms / 1e3)
            out["popcount"] = dict(value=prate, ms_per_step=pms, kernel_ms=pkms)
            out["mfma_over_popcount"] = rate / prate
            if "mfma_int8" in out:
                out["mfma_int8_over_popcount"] = out["mfma_int8"]["value"] / prate
    else:
        out["roofline"] = dict(bound="alu", achieved=None, peak=None, unit=None, frac=None,
                               traffic=None, kernel="pop2_kernel", kernel_ms=kms)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_2way(args, v, n_f)
    return out


def bench_3way(args, lib, missing, workload):
    import torch
    import paper_1705_08213_amd as ccc
    import synth
    n_v, n_f = 2048, 16384
    log(f"generating {n_v} x {n_f} input")
    v = synth.beta_hw(n_v, n_f, seed=0, missing=missing)
    dv = torch.from_numpy(v).cuda()
    T = ccc.n_triples(n_v)
    tables = torch.empty((T, 8), dtype=torch.int32, device="cuda")
    cc = torch.empty((T, 8), dtype=torch.float64, device="cuda")
    counts = torch.empty((n_v, 4), dtype=torch.int32, device="cuda")

    def step():
        ccc.ccc_3way(dv, n_f, tables, cc, counts, path="mfma", operands=args.operands)

    ms, kms, _ = timed(step, args.steps, args.warmup, lib, "mfma3")
    comps = T * n_f
    # 8 MACs per comparison; with no missing entry every unit takes the
    # one-plane complete-data form (1 MAC per comparison)
    fmt, peak, dt = mfma_format(n_f, args.operands)
    ops_per = 2.0 if missing == 0.0 else 16.0
    ach = ops_per * comps / (kms / 1e3) / 1e12
    alg_bytes = n_v * ((n_f + 3) // 4) + 96 * T + 16 * n_v
    roof = dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                frac=ach / peak, traffic=None,
                traffic_unit="bytes per launch (FETCH_SIZE+WRITE_SIZE, scaled)",
                algorithmic_bytes=alg_bytes,
                kernel=("mfma3_complete_kernel" if missing == 0.0 else "mfma3_run_kernel")
                if fmt == "fp4" else "mfma3_kernel", kernel_ms=kms,
                operands=fmt, ops_per_comparison=int(ops_per))
    if fmt == "fp4":
        roof["traffic"] = committed_traffic(
            MFMA3_SOURCES, "profiles/mfma3_3way_n2048_f16384.md" if missing > 0.0
            else "profiles/mfma3_3way_complete_n2048_f16384.md")
    hbm = alg_bytes / (kms / 1e3) / 1e9
    if hbm / HBM_PEAK_GBS > roof["frac"]:
        # the output stream, not the matrix cores, is the nearer ceiling
        roof.update(bound="hbm", achieved=hbm, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=hbm / HBM_PEAK_GBS, mfma_frac=ach / peak)
    out = dict(metric="CCC comparisons/sec (triples*n_f), bit-exact tables",
               value=comps / (ms / 1e3), unit="comparisons/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype=dt, data="synthetic",
               config=dict(workload=workload, n_v=n_v, n_f=n_f, missing=missing, path="mfma",
                           operands=fmt),
               roofline=roof)
    if args.select_threshold is not None:
        thr = args.select_threshold
        found = {}

        def sel_step():
            found["n"] = ccc.ccc_3way_select(dv, n_f, thr, cap=1 << 22, counts=counts)[0]

        sms, _, _ = timed(sel_step, args.steps, 1, lib, "mfma3")
        out["select"] = dict(threshold=thr, kept=found["n"], ms_per_step=sms,
                             value=comps / (sms / 1e3),
                             note="ccc_3way_select: only triples with a CCC value >= threshold "
                                  "are written (includes a count read-back)")
    if args.pop_steps > 0:
        log(f"timing popcount 3-way: 1 warmup + {args.pop_steps} steps")

        def pop_step():
            ccc.ccc_3way(dv, n_f, tables, cc, counts, path="popcount")

        pms, pkms, _ = timed(pop_step, args.pop_steps, 1, lib, "pop3")
        out["popcount"] = dict(value=comps / (pms / 1e3), ms_per_step=pms, kernel_ms=pkms)
        out["mfma_over_popcount"] = pms / ms
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_3way(args, v, n_f)
    return out


def bench_multi(args, lib):
    import torch
    import paper_1705_08213_amd as ccc
    import synth
    n_v, n_f, s, missing = 16384, 32768, 4, 0.01
    log(f"generating {n_v} x {n_f} multi-allelic input, s = {s}")
    v = synth.multi_hw(n_v, n_f, s, seed=0, missing=missing)
    dv = torch.from_numpy(v).cuda()
    P = ccc.n_pairs(n_v)
    tables = torch.empty((P, s * s), dtype=torch.int32, device="cuda")
    cc = torch.empty((P, s * s), dtype=torch.float64, device="cuda")
    counts = torch.empty((n_v, 8), dtype=torch.int32, device="cuda")

    def step():
        ccc.ccc_2way_multi(dv, n_f, s, tables, cc, counts, operands=args.operands)

    ms, kms, _ = timed(step, args.steps, args.warmup, lib, "multi2")
    comps = P * n_f
    ops = 2.0 * s * s * comps  # s^2 MACs per comparison
    ach = ops / (kms / 1e3) / 1e12
    fmt, peak, dt = mfma_format(n_f, args.operands)
    out = dict(metric="CCC comparisons/sec (pairs*n_f), bit-exact tables", value=comps / (ms / 1e3),
               unit="comparisons/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype=dt, data="synthetic",
               config=dict(workload=f"2-way multi-allelic CCC: n_v={n_v} x n_f={n_f}, s={s} "
                                    "states, normalised sin^2 frequencies / Hardy-Weinberg, "
                                    "1% missing", n_v=n_v, n_f=n_f, states=s, missing=missing,
                           path="mfma", operands=fmt),
               roofline=dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                             frac=ach / peak, operands=fmt,
                             traffic=committed_traffic(MULTI2_SOURCES,
                                                       "profiles/multi2_2way_n16384_f32768_s4.md")
                             if fmt == "fp4" else None,
                             traffic_unit="bytes per launch (FETCH_SIZE+WRITE_SIZE, scaled)",
                             algorithmic_bytes=n_v * n_f + P * s * s * 12 + 32 * n_v,
                             kernel="multi2_kernel", kernel_ms=kms,
                             ops_per_comparison=int(2 * s * s)))
    if not args.no_cpu:
        import oracle
        pairs = lambda r0, r1: sum(n_v - 1 - i for i in range(r0, r1))
        out["cpu_baseline"] = cpu_baseline(
            args, lambda r0, r1: oracle.multi_two_way(v, n_f, s, r0, r1),
            lambda r0, r1: pairs(r0, r1) * n_f, n_v, P * n_f, "pairs (i, j > i)")
    return out


def bench_block(args, lib):
    import torch
    import paper_1705_08213_amd as ccc
    import synth
    n, n_f, chunk, missing = 16384, 131072, 16384, 0.02
    log(f"generating 2 x {n} x {n_f} input")
    ha = synth.beta_hw(n, n_f, seed=0, missing=missing)
    hb = synth.beta_hw(n, n_f, seed=1, missing=missing)
    va, vb = torch.from_numpy(ha).cuda(), torch.from_numpy(hb).cuda()
    tables = torch.empty((n, n, 4), dtype=torch.int32, device="cuda")
    cc = torch.empty((n, n, 4), dtype=torch.float64, device="cuda")
    ca = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    cb = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    nchunks = n_f // chunk

    def step():
        for k in range(nchunks):
            ccc.ccc_2way_block(va, vb, chunk, tables, ca, cb, cc, accumulate=k > 0,
                               finalize=k == nchunks - 1, field_offset=k * chunk // 4,
                               operands=args.operands)

    ms, kms, kn = timed(step, args.steps, args.warmup, lib, "mfma2")
    comps = n * n * n_f
    per_launch = 8.0 * n * n * chunk
    ach = per_launch / (kms / 1e3) / 1e12
    fmt, peak, dt = mfma_format(chunk, args.operands)
    out = dict(metric="CCC comparisons/sec (n_a*n_b*n_f), bit-exact tables",
                value=comps / (ms / 1e3), unit="comparisons/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=ms, higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype=dt, data="synthetic",
                config=dict(workload="2-way block 16384 x 16384, n_f=131072 in 8 chunks of "
                                     "16384, Beta/HW, 2% missing", path="mfma", operands=fmt),
                roofline=dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                              frac=ach / peak, traffic=None, kernel="mfma2_kernel",
                              kernel_ms=kms, operands=fmt))
    if not args.no_cpu:
        import oracle
        del va, vb, tables, cc
        out["cpu_baseline"] = cpu_baseline(
            args, lambda r0, r1: oracle.block(ha, hb, n_f, r0, r1, with_ccc=True),
            lambda r0, r1: (r1 - r0) * n * n_f, n, comps, "pairs (i in A, all j in B)")
    return out


def bench_many(args, lib):
    import torch
    import paper_1705_08213_amd as ccc
    import synth
    nv, nf = synth.batch_sizes(64, seed=0)
    log(f"generating 64 problems, sum n_v = {int(nv.sum())}")
    probs, hosts = [], []
    comps = 0
    for k in range(64):
        v = synth.beta_hw(int(nv[k]), int(nf[k]), seed=100 + k, missing=0.01)
        hosts.append(v)
        probs.append(dict(v=torch.from_numpy(v).cuda(), n_f=int(nf[k])))
        comps += ccc.n_pairs(int(nv[k])) * int(nf[k])
    for p in probs:  # outputs allocated up front, as a serving caller would
        n_v = p["v"].shape[0]
        P = ccc.n_pairs(n_v)
        p.update(tables=torch.empty((P, 4), dtype=torch.int32, device="cuda"),
                 ccc=torch.empty((P, 4), dtype=torch.float64, device="cuda"),
                 counts=torch.empty((n_v, 4), dtype=torch.int32, device="cuda"))
    # first call: work list, upload, graph capture and instantiation (host
    # time the library records as "many_setup"), then the first replay
    torch.cuda.synchronize()
    lib.ccc_timing_reset()
    lib.ccc_timing_enable(1)
    t0 = time.perf_counter()
    ccc.ccc_2way_many(probs, operands=args.operands)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    lib.ccc_timing_enable(0)
    setup_ms, _ = timing_query(lib, "many_setup")
    lib.ccc_timing_reset()

    def step():
        ccc.ccc_2way_many(probs, operands=args.operands)

    ms, kms, kn = timed(step, args.steps, args.warmup, lib, "many")
    fmt, peak, dt = mfma_format(int(nf.max()), args.operands)
    out = dict(metric="CCC comparisons/sec (sum pairs*n_f), bit-exact tables",
                value=comps / (ms / 1e3), unit="comparisons/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=ms, higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype=dt, data="synthetic",
                config=dict(workload="64 batched 2-way problems, n_v log-uniform [256,8192], "
                                     "n_f uniform [1000,50000], Beta/HW, 1% missing",
                            path="mfma", operands=fmt),
                roofline=dict(bound="mfma", achieved=8.0 * comps / (kms / 1e3) / 1e12,
                              peak=peak, unit="TFLOP/s",
                              frac=8.0 * comps / (kms / 1e3) / 1e12 / peak,
                              traffic=None, kernel="graph replay (count + persistent tally "
                                                   "launches)", kernel_ms=kms, operands=fmt),
                graph=dict(setup_ms=setup_ms, first_call_ms=first_ms,
                           note="setup_ms: host time of the work list, its upload, graph "
                                "capture and instantiation on first sight of the batch; "
                                "first_call_ms adds the first replay and a sync"))
    if not args.no_cpu:
        import oracle
        # rows [8 c0, 8 c1) of every problem
        def call(c0, c1):
            for v, f in zip(hosts, nf):
                if 8 * c0 < v.shape[0]:
                    oracle.two_way(v, int(f), 8 * c0, min(8 * c1, v.shape[0]), with_ccc=True)

        def comps_of(c0, c1):
            tot = 0
            for n_v, f in zip(nv, nf):
                n_v = int(n_v)
                for i in range(8 * c0, min(8 * c1, n_v)):
                    tot += (n_v - 1 - i) * int(f)
            return tot

        out["cpu_baseline"] = cpu_baseline(args, call, comps_of, (int(nv.max()) + 7) // 8, comps,
                                           "pairs of every problem (rows x 8)", chunk=1)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pop-steps", type=int, default=2,
                    help="popcount-path steps (c2, c2c, c3, c3c)")
    ap.add_argument("--config", default="c2",
                    choices=["c1", "c2", "c2c", "c2m", "c3", "c3c", "c4", "c5"])
    ap.add_argument("--operands", default="auto", choices=["auto", "fp4", "int8"],
                    help="MFMA operand format (auto: fp4 while n_f <= 2^22, int8 beyond)")
    ap.add_argument("--other-steps", type=int, default=5,
                    help="steps of the same 2-way call with the other operand format (c2, c2c)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-comparisons", type=float, default=1e11,
                    help="comparisons the all-threads oracle sample aims for")
    ap.add_argument("--cpu-seconds", type=float, default=30.0,
                    help="time limit of the all-threads oracle sample (whole row chunks)")
    ap.add_argument("--cpu-one-core-seconds", type=float, default=5.0,
                    help="time of the one-thread oracle sample (0: skip it)")
    ap.add_argument("--select-threshold", type=float, default=None,
                    help="also time the threshold-filtered entry point (c2, c3); e.g. 0.13 "
                         "for 2-way, 0.05 for 3-way (independent vectors stay below 0.141 and "
                         "0.053)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain elementwise copy of 1 GiB (read 1 GiB, write 1 GiB) "
                         "to scale the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps(dict(error="this benchmark runs on exactly one GPU; the library "
                                    "has no multi-GPU sharding", n_gpus=args.gpus)))
        sys.exit(2)
    import torch
    import paper_1705_08213_amd as ccc
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1, out=b)
        torch.cuda.synchronize()
        print(json.dumps(dict(calibration="elementwise int32 add, 2^28 elements: reads 1 GiB, "
                                          "writes 1 GiB per launch", launches=3)))
        return
    lib = ccc.lib()
    lib.ccc_timing_enable.argtypes = [ctypes.c_int]
    if args.config == "c2":
        out = bench_2way(args, lib, 32768, 65536, 0.01, "beta_hw", "mfma",
                         "2-way CCC large: n_v=32768 x n_f=65536, Beta(0.5,0.5)/Hardy-Weinberg, "
                         "1% missing")
    elif args.config == "c2c":
        out = bench_2way(args, lib, 32768, 65536, 0.0, "beta_hw", "mfma",
                         "2-way CCC, complete data: n_v=32768 x n_f=65536, "
                         "Beta(0.5,0.5)/Hardy-Weinberg, no missing")
    elif args.config == "c1":
        out = bench_2way(args, lib, 512, 1000, 0.0, "uniform", "popcount",
                         "2-way CCC: n_v=512 x n_f=1000, uniform genotypes, no missing")
    elif args.config == "c3":
        out = bench_3way(args, lib, 0.005, "3-way CCC: n_v=2048 x n_f=16384, "
                                           "Beta(0.5,0.5)/Hardy-Weinberg, 0.5% missing")
    elif args.config == "c3c":
        out = bench_3way(args, lib, 0.0, "3-way CCC, complete data: n_v=2048 x n_f=16384, "
                                         "Beta(0.5,0.5)/Hardy-Weinberg, no missing")
    elif args.config == "c4":
        out = bench_many(args, lib)
    elif args.config == "c2m":
        out = bench_multi(args, lib)
    else:
        out = bench_block(args, lib)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
