"""Autotuner for the 2-way MFMA launches: picks the tile variant (and, for the
batched launch, the persistent workgroups per compute unit) per size class
and writes the table the library reads.

    python -m paper_1705_08213_amd.tune [--out paper_1705_08213_amd/tune_gfx950.txt]
                                        [--summary sweep.md]

Batched (``ccc_2way_many``, kind ``mfma``): for every size class (n_v up to a
bound, n_f up to a bound) it builds a batch of problems with sizes spread
over the class and times the batch with each tile variant and workgroups-per-
CU figure forced through ``CCC_MANY_VARIANT`` / ``CCC_MANY_WG`` (graph built
on the first call, replays timed).

One-shot (``ccc_2way``, kind ``oneshot``): for every size class it times one
representative problem with each variant forced through
``CCC_ONESHOT_VARIANT``.

The fastest choice of each class becomes a line ``n_v_max n_f_max kind
variant [wg_per_cu]``.  Inputs are random packed bytes made on the device:
the kernels' execution path does not depend on the values beyond the
complete-data vote, which random codes (a quarter of them missing) fail.
The summary (Markdown) lists every timing of the sweep.
"""
from __future__ import annotations

import argparse
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# (n_v_max, n_f_max) classes, matched first-to-last by the library
MANY_CLASSES = [(384, 8192), (384, 1 << 29), (1024, 8192), (1024, 1 << 29), (3072, 8192),
                (3072, 1 << 29), (1 << 30, 1 << 29)]
# batched tile variants (workgroup tile) and the workgroups per CU each may use
MANY_VARIANTS = {0: "128x64", 1: "64x32", 2: "64x64", 3: "32x32"}
MANY_MAX_WG = {0: 2, 1: 4, 2: 2, 3: 4}
WG_CHOICES = (1, 2, 3, 4)

ONESHOT_CLASSES = [(384, 8192), (384, 1 << 29), (1024, 8192), (1024, 1 << 29), (3072, 8192),
                   (3072, 1 << 29), (8192, 8192), (8192, 1 << 29), (1 << 30, 1 << 29)]
ONESHOT_VARIANTS = {0: "128x64", 1: "64x32", 2: "64x64"}


def packed(n_v, n_f, gen):
    import torch
    ld = max(16, ((n_f + 3) // 4 + 15) // 16 * 16)
    return torch.randint(0, 256, (n_v, ld), dtype=torch.uint8, device="cuda", generator=gen)


def class_batch(nv_lo, nv_hi, nf_lo, nf_hi, count, gen):
    probs = []
    for k in range(count):
        t = (k + 0.5) / count
        n_v = int(math.exp(math.log(nv_lo) + t * (math.log(nv_hi) - math.log(nv_lo))))
        n_f = int(nf_lo + ((k * 7) % count + 0.5) / count * (nf_hi - nf_lo))
        probs.append(dict(v=packed(n_v, n_f, gen), n_f=n_f))
    return probs


def elapsed_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def with_env(env, fn):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return fn()
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def time_many(probs, variant, wg, reps=5):
    from paper_1705_08213_amd import ccc_2way_many

    def run():
        outs = ccc_2way_many(probs)
        batch = [dict(p, tables=t, ccc=c, counts=cnt) for p, (t, c, cnt) in zip(probs, outs)]
        return elapsed_ms(lambda: ccc_2way_many(batch), reps)
    return with_env({"CCC_MANY_VARIANT": variant, "CCC_MANY_WG": wg}, run)


def time_oneshot(v, n_f, variant, reps=3):
    import torch
    from paper_1705_08213_amd import ccc_2way, n_pairs
    n_v = v.shape[0]
    P = n_pairs(n_v)
    t = torch.empty((P, 4), dtype=torch.int32, device="cuda")
    c = torch.empty((P, 4), dtype=torch.float64, device="cuda")
    cnt = torch.empty((n_v, 4), dtype=torch.int32, device="cuda")
    return with_env({"CCC_ONESHOT_VARIANT": variant},
                    lambda: elapsed_ms(lambda: ccc_2way(v, n_f, t, c, cnt), reps))


def class_ranges(classes, nv_floor, nv_cap, nf_cap):
    """(nv_lo, nv_hi, nf_lo, nf_hi) spanned by each class (matched first to
    last: a class starts above the previous bound on its axis)."""
    out, prev_nv, nv_lo = [], None, nv_floor
    for nv_max, nf_max in classes:
        if prev_nv is not None and nv_max != prev_nv:
            nv_lo = prev_nv + 1
        lo_nf, hi_nf = (8193, min(nf_max, nf_cap)) if nf_max > 8192 else (256, nf_max)
        out.append((max(nv_lo, nv_floor), min(nv_max, nv_cap), lo_nf, hi_nf))
        prev_nv = nv_max
    return out


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tune_gfx950.txt"))
    ap.add_argument("--summary", default=None, help="write the sweep's timings (Markdown)")
    ap.add_argument("--problems", type=int, default=12)
    args = ap.parse_args()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    lines = ["# 2-way MFMA tile shapes per size class on gfx950, written by "
             "paper_1705_08213_amd/tune.py",
             "# n_v_max n_f_max kind variant [wg_per_cu]",
             "# mfma (ccc_2way_many) variants: " +
             ", ".join(f"{k} = {v}" for k, v in MANY_VARIANTS.items()) + " workgroup tiles",
             "# oneshot (ccc_2way, _rows, _select, _block) variants: " +
             ", ".join(f"{k} = {v}" for k, v in ONESHOT_VARIANTS.items())]
    md = ["# 2-way MFMA tile-shape sweep (gfx950)", "",
          "Command: `python -m paper_1705_08213_amd.tune --summary <this file>` "
          "(random packed inputs, times in ms, fastest marked *).", "",
          "## Batched (`ccc_2way_many`): one batch of "
          f"{args.problems} problems per class, variant x workgroups per CU", ""]
    choices = [(v, wg) for v in MANY_VARIANTS for wg in WG_CHOICES if wg <= MANY_MAX_WG[v]]
    md.append("| class (n_v, n_f) | " + " | ".join(f"{MANY_VARIANTS[v]} wg{wg}"
                                                 for v, wg in choices) + " |")
    md.append("|---|" + "---|" * len(choices))
    for (nv_max, nf_max), (lo_nv, hi_nv, lo_nf, hi_nf) in zip(
            MANY_CLASSES, class_ranges(MANY_CLASSES, 64, 8192, 50000)):
        probs = class_batch(lo_nv, hi_nv, lo_nf, hi_nf, args.problems, gen)
        times = {c: time_many(probs, *c) for c in choices}
        best = min(times, key=times.get)
        print(f"many n_v<={nv_max} n_f<={nf_max}: " +
              ", ".join(f"{MANY_VARIANTS[v]}/wg{wg} {t:.3f}" for (v, wg), t in times.items()) +
              f" -> {best}", flush=True)
        lines.append(f"{nv_max} {nf_max} mfma {best[0]} {best[1]}")
        md.append(f"| {lo_nv}..{hi_nv}, {lo_nf}..{hi_nf} | " +
                  " | ".join(f"{times[c]:.3f}" + ("*" if c == best else "") for c in choices) +
                  " |")
        del probs
        torch.cuda.empty_cache()
    md += ["", "## One-shot (`ccc_2way`): one problem per class (geometric middle of the "
           "class's n_v, n_f 4096 or 32768)", "",
           "| class | problem | " + " | ".join(ONESHOT_VARIANTS.values()) + " |",
           "|---|---|" + "---|" * len(ONESHOT_VARIANTS)]
    for (nv_max, nf_max), (lo_nv, hi_nv, _, _) in zip(
            ONESHOT_CLASSES, class_ranges(ONESHOT_CLASSES, 64, 16384, 1 << 29)):
        n_v = int(math.sqrt(lo_nv * hi_nv))
        n_f = 4096 if nf_max <= 8192 else 32768
        v = packed(n_v, n_f, gen)
        times = {var: time_oneshot(v, n_f, var) for var in ONESHOT_VARIANTS}
        best = min(times, key=times.get)
        print(f"oneshot n_v<={nv_max} n_f<={nf_max} ({n_v} x {n_f}): " +
              ", ".join(f"{ONESHOT_VARIANTS[k]} {t:.3f}" for k, t in times.items()) +
              f" -> {best}", flush=True)
        lines.append(f"{nv_max} {nf_max} oneshot {best}")
        md.append(f"| n_v <= {nv_max}, n_f <= {nf_max} | {n_v} x {n_f} | " +
                  " | ".join(f"{times[k]:.3f}" + ("*" if k == best else "")
                             for k in ONESHOT_VARIANTS) + " |")
        del v
        torch.cuda.empty_cache()
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", args.out)
    if args.summary:
        with open(args.summary, "w") as f:
            f.write("\n".join(md) + "\n")
        print("wrote", args.summary)


if __name__ == "__main__":
    main()
