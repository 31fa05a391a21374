#!/usr/bin/env python3
"""Throughput of the CCC tally hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]

A step is one call of the library's entry point for the workload (1-way
count pass, tally kernel and fused FP64 epilogue writing every table and CCC
value) on inputs already resident in HBM.  The default workload is the large
2-way configuration (n_v = 32768 vectors x n_f = 65536 fields, per-vector
allele frequency ~ Beta(1/2,1/2), Hardy-Weinberg genotypes, 1% missing) on
the int8-MFMA path; the popcount path is timed on the same input for the
ratio.  Prints one JSON line.

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


def mfma_format(n_f):
    """(operand format, dense peak in T(FL)OP/s, dtype tag) of the MFMA kernels
    over n_f fields, as the library reports it."""
    import paper_1705_08213_amd as ccc
    fmt = ccc.mfma_operands(n_f)
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


def oracle_sample(call, units, n_rows, chunk, seconds):
    """Runs call(r0, r1) over consecutive row chunks from row 0 until `seconds`
    of CPU time have passed (at least one chunk) or the rows run out; returns
    (rows, units, s)."""
    rows, done, dt = 0, 0, 0.0
    while rows < n_rows and (rows == 0 or dt < seconds):
        r1 = min(n_rows, rows + chunk)
        t = time.perf_counter()
        call(rows, r1)
        dt += time.perf_counter() - t
        done += sum(units(i) for i in range(rows, r1))
        rows = r1
    return rows, done, dt


def cpu_baseline_2way(v, n_f, seconds):
    """The oracle on rows [0, rows) x all later vectors (plain loops, OpenMP)."""
    import oracle
    n_v = v.shape[0]
    rows, pairs, dt = oracle_sample(
        lambda r0, r1: oracle.two_way(v, n_f, r0, r1, with_ccc=True),
        lambda i: n_v - 1 - i, n_v, 8, seconds)
    return dict(value=pairs * n_f / dt, unit="comparisons/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"rows i in [0,{rows}) x all j>i of the same input ({pairs} pairs x "
                       f"{n_f} fields, {dt:.1f} s)")


def cpu_baseline_3way(v, n_f, seconds):
    import oracle
    n_v = v.shape[0]
    rows, tri, dt = oracle_sample(
        lambda r0, r1: oracle.three_way(v, n_f, r0, r1, with_ccc=True),
        lambda i: (n_v - 1 - i) * (n_v - 2 - i) // 2, n_v, 1, seconds)
    return dict(value=tri * n_f / dt, unit="comparisons/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"triples with i in [0,{rows}) of the same input ({tri} triples x "
                       f"{n_f} fields, {dt:.1f} s)")


def bench_2way(args, lib, n_v, n_f, missing, gen, path, workload, cpu_seconds):
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

    def step(p=path):
        ccc.ccc_2way(dv, n_f, tables, cc, counts, path=p)

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
        fmt, peak, _ = mfma_format(n_f)
        out["config"]["operands"] = fmt
        ops = (2.0 if missing == 0.0 else 8.0) * comps
        ach = ops / (kms / 1e3) / 1e12
        traffic = None
        if (n_v, n_f) == (32768, 65536):
            traffic = committed_traffic(
                MFMA2_SOURCES, "profiles/mfma2_2way_n32768_f65536_traffic.md" if missing > 0.0
                else "profiles/mfma2_2way_complete_n32768_f65536.md")
        out["roofline"] = dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                               frac=ach / peak, traffic=traffic,
                               traffic_unit="bytes per launch (FETCH_SIZE+WRITE_SIZE, scaled)",
                               algorithmic_bytes=n_v * ((n_f + 3) // 4) + 48 * P + 32 * n_v,
                               kernel="mfma2_kernel", kernel_ms=kms, operands=fmt,
                               ops_per_comparison=2 if missing == 0.0 else 8,
                               frac_of_int8_peak=ach / INT8_PEAK_TOPS)
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
    else:
        out["roofline"] = dict(bound="alu", achieved=None, peak=None, unit=None, frac=None,
                               traffic=None, kernel="pop2_kernel", kernel_ms=kms)
    if not args.no_cpu:
        log(f"timing the CPU oracle for about {cpu_seconds:g} s")
        out["cpu_baseline"] = cpu_baseline_2way(v, n_f, cpu_seconds)
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
        ccc.ccc_3way(dv, n_f, tables, cc, counts, path="mfma")

    ms, kms, _ = timed(step, args.steps, args.warmup, lib, "mfma3")
    comps = T * n_f
    # 8 MACs per comparison; with no missing entry every unit takes the
    # one-plane complete-data form (1 MAC per comparison)
    fmt, peak, dt = mfma_format(n_f)
    ops_per = 2.0 if missing == 0.0 else 16.0
    ach = ops_per * comps / (kms / 1e3) / 1e12
    alg_bytes = n_v * ((n_f + 3) // 4) + 96 * T + 16 * n_v
    roof = dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                frac=ach / peak, traffic=None,
                traffic_unit="bytes per launch (FETCH_SIZE+WRITE_SIZE, scaled)",
                algorithmic_bytes=alg_bytes, kernel="mfma3_kernel", kernel_ms=kms,
                operands=fmt, ops_per_comparison=int(ops_per),
                frac_of_int8_peak=ach / INT8_PEAK_TOPS)
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
        out["cpu_baseline"] = cpu_baseline_3way(v, n_f, args.cpu_seconds)
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
        ccc.ccc_2way_multi(dv, n_f, s, tables, cc, counts)

    ms, kms, _ = timed(step, args.steps, args.warmup, lib, "multi2")
    comps = P * n_f
    ops = 2.0 * s * s * comps  # s^2 MACs per comparison
    ach = ops / (kms / 1e3) / 1e12
    fmt, peak, dt = mfma_format(n_f)
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
                                                       "profiles/multi2_2way_n16384_f32768_s4.md"),
                             traffic_unit="bytes per launch (FETCH_SIZE+WRITE_SIZE, scaled)",
                             algorithmic_bytes=n_v * n_f + P * s * s * 12 + 32 * n_v,
                             kernel="multi2_kernel", kernel_ms=kms,
                             ops_per_comparison=int(2 * s * s),
                             frac_of_int8_peak=ach / INT8_PEAK_TOPS))
    if not args.no_cpu:
        import oracle
        rows, pairs, dt = oracle_sample(lambda r0, r1: oracle.multi_two_way(v, n_f, s, r0, r1),
                                        lambda i: n_v - 1 - i, n_v, 8, args.cpu_seconds)
        out["cpu_baseline"] = dict(value=pairs * n_f / dt, unit="comparisons/s",
                                   cores=oracle.num_threads(), kind="oracle",
                                   sample=f"rows i in [0,{rows}) x all j>i of the same input "
                                          f"({pairs} pairs x {n_f} fields, {dt:.1f} s)")
    return out


def bench_block(args, lib):
    import torch
    import paper_1705_08213_amd as ccc
    import synth
    n, n_f, chunk, missing = 16384, 131072, 16384, 0.02
    log(f"generating 2 x {n} x {n_f} input")
    va = torch.from_numpy(synth.beta_hw(n, n_f, seed=0, missing=missing)).cuda()
    vb = torch.from_numpy(synth.beta_hw(n, n_f, seed=1, missing=missing)).cuda()
    tables = torch.empty((n, n, 4), dtype=torch.int32, device="cuda")
    cc = torch.empty((n, n, 4), dtype=torch.float64, device="cuda")
    ca = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    cb = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    nchunks = n_f // chunk

    def step():
        for k in range(nchunks):
            ccc.ccc_2way_block(va, vb, chunk, tables, ca, cb, cc, accumulate=k > 0,
                               finalize=k == nchunks - 1, field_offset=k * chunk // 4)

    ms, kms, kn = timed(step, args.steps, args.warmup, lib, "mfma2")
    comps = n * n * n_f
    per_launch = 8.0 * n * n * chunk
    ach = per_launch / (kms / 1e3) / 1e12
    fmt, peak, dt = mfma_format(chunk)
    return dict(metric="CCC comparisons/sec (n_a*n_b*n_f), bit-exact tables",
                value=comps / (ms / 1e3), unit="comparisons/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=ms, higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype=dt, data="synthetic",
                config=dict(workload="2-way block 16384 x 16384, n_f=131072 in 8 chunks of "
                                     "16384, Beta/HW, 2% missing", path="mfma", operands=fmt),
                roofline=dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
                              frac=ach / peak, traffic=None, kernel="mfma2_kernel",
                              kernel_ms=kms, operands=fmt))


def bench_many(args, lib):
    import torch
    import paper_1705_08213_amd as ccc
    import synth
    nv, nf = synth.batch_sizes(64, seed=0)
    log(f"generating 64 problems, sum n_v = {int(nv.sum())}")
    probs = []
    comps = 0
    for k in range(64):
        v = synth.beta_hw(int(nv[k]), int(nf[k]), seed=100 + k, missing=0.01)
        probs.append(dict(v=torch.from_numpy(v).cuda(), n_f=int(nf[k])))
        comps += ccc.n_pairs(int(nv[k])) * int(nf[k])
    outs = ccc.ccc_2way_many(probs)
    for p, (t, c, cnt) in zip(probs, outs):
        p.update(tables=t, ccc=c, counts=cnt)

    def step():
        ccc.ccc_2way_many(probs)

    ms, kms, kn = timed(step, args.steps, args.warmup, lib, "mfma2")
    fmt, peak, dt = mfma_format(int(nf.max()))
    return dict(metric="CCC comparisons/sec (sum pairs*n_f), bit-exact tables",
                value=comps / (ms / 1e3), unit="comparisons/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=ms, higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype=dt, data="synthetic",
                config=dict(workload="64 batched 2-way problems, n_v log-uniform [256,8192], "
                                     "n_f uniform [1000,50000], Beta/HW, 1% missing",
                            path="mfma", operands=fmt),
                roofline=dict(bound="mfma", achieved=8.0 * comps / (ms / 1e3) / 1e12,
                              peak=peak, unit="TFLOP/s",
                              frac=8.0 * comps / (ms / 1e3) / 1e12 / peak,
                              traffic=None, kernel="whole step", operands=fmt))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pop-steps", type=int, default=2,
                    help="popcount-path steps (c2, c2c, c3, c3c)")
    ap.add_argument("--config", default="c2",
                    choices=["c1", "c2", "c2c", "c2m", "c3", "c3c", "c4", "c5"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU time the oracle baseline runs for (whole row chunks)")
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
                         "1% missing", args.cpu_seconds)
    elif args.config == "c2c":
        out = bench_2way(args, lib, 32768, 65536, 0.0, "beta_hw", "mfma",
                         "2-way CCC, complete data: n_v=32768 x n_f=65536, "
                         "Beta(0.5,0.5)/Hardy-Weinberg, no missing", args.cpu_seconds)
    elif args.config == "c1":
        out = bench_2way(args, lib, 512, 1000, 0.0, "uniform", "popcount",
                         "2-way CCC: n_v=512 x n_f=1000, uniform genotypes, no missing",
                         args.cpu_seconds)
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
