"""Autotuner for the batched 2-way path (``ccc_2way_many``): picks the tile
variant per size class and writes the table the library reads.

    python -m paper_1705_08213_amd.tune [--out paper_1705_08213_amd/tune_gfx950.txt]

For every size class (n_v up to a bound, n_f up to a bound) it builds a batch
of problems with sizes spread over the class, times ``ccc_2way_many`` with
each tile variant forced through ``CCC_MANY_VARIANT`` (graph built on the
first call, replays timed), and writes the fastest variant as a line
``n_v_max n_f_max mfma variant``.  Inputs are random packed bytes made on the
device: the kernels' execution path does not depend on the values.
"""
from __future__ import annotations

import argparse
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# (n_v_max, n_f_max) classes, matched first-to-last by the library
CLASSES = [(384, 8192), (384, 1 << 29), (1024, 8192), (1024, 1 << 29), (3072, 8192),
           (3072, 1 << 29), (1 << 30, 1 << 29)]
VARIANTS = (0, 1)


def class_batch(nv_lo, nv_hi, nf_lo, nf_hi, count, gen):
    import torch
    probs = []
    for k in range(count):
        t = (k + 0.5) / count
        n_v = int(math.exp(math.log(nv_lo) + t * (math.log(nv_hi) - math.log(nv_lo))))
        n_f = int(nf_lo + ((k * 7) % count + 0.5) / count * (nf_hi - nf_lo))
        ld = max(16, ((n_f + 3) // 4 + 15) // 16 * 16)
        v = torch.randint(0, 256, (n_v, ld), dtype=torch.uint8, device="cuda", generator=gen)
        probs.append(dict(v=v, n_f=n_f))
    return probs


def time_variant(probs, variant, reps=5):
    import torch
    from paper_1705_08213_amd import ccc_2way_many
    os.environ["CCC_MANY_VARIANT"] = str(variant)
    try:
        outs = ccc_2way_many(probs)
        batch = [dict(p, tables=t, ccc=c, counts=cnt) for p, (t, c, cnt) in zip(probs, outs)]
        ccc_2way_many(batch)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ccc_2way_many(batch)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        del os.environ["CCC_MANY_VARIANT"]


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tune_gfx950.txt"))
    ap.add_argument("--problems", type=int, default=12)
    args = ap.parse_args()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    lines = ["# ccc_2way_many tile variant per size class on gfx950, written by "
             "paper_1705_08213_amd/tune.py",
             "# n_v_max n_f_max path variant   (variant 0: 128x64 workgroup tiles, "
             "1: 64x32)"]
    nv_lo, prev_nv = 2, None
    for nv_max, nf_max in CLASSES:
        if prev_nv is not None and nv_max != prev_nv:
            nv_lo = prev_nv + 1
        lo_nv, hi_nv = max(nv_lo, 64), min(nv_max, 8192)
        lo_nf = 1000 if nf_max > 8192 else 256
        hi_nf = min(nf_max, 50000)
        if nf_max > 8192:
            lo_nf = 8193
        probs = class_batch(lo_nv, hi_nv, lo_nf, hi_nf, args.problems, gen)
        times = {v: time_variant(probs, v) for v in VARIANTS}
        best = min(times, key=times.get)
        print(f"class n_v<={nv_max} n_f<={nf_max}: " +
              ", ".join(f"variant {v}: {t:.3f} ms" for v, t in times.items()) + f" -> {best}",
              flush=True)
        lines.append(f"{nv_max} {nf_max} mfma {best}")
        prev_nv = nv_max
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", args.out)


if __name__ == "__main__":
    main()
