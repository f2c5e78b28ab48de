"""Time the candidate schedules of every shape on the device and write the table
that the library's automatic schedule reads (csrc/schedule_table.inc).

A key is (precision, coupled waves, log2 nt, alone or in a batch). For each key
the candidates are the distinct four-step splits (log2 of the column length) of
the two-pass kernels and, where the shape is served, the resident
pass. Each candidate runs CW singly resonant oscillators of that shape: one
instance alone, or a batch of same-shape instances that fills the chip (about
2^22 points, from two to 512 instances). In a batch only splits that the default
split's column and row kernels serve are candidates, so that any mix of batched
shapes keeps the paired (mixed) launches. Each timing is the best of three
windows of about 30 ms. The timing is taken here, once, on the
target device; the library only looks the result up, so the same shape always
gets the same schedule (no timing-dependent rounding at run time). The fastest
candidate of a key wins unless it is within 2 % of the default schedule, which
then stays.

Usage (needs the GPU): python -m paper_2410_02532_amd.tune [--out FILE] [--summary FILE]
"""
import argparse
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2410_02532_amd import opo as B          # noqa: E402
from paper_2410_02532_amd import workloads as W    # noqa: E402

MAX_LOG2 = {"f32": 20, "f64": 19}
MAX_LOG2_N1 = {"f32": 12, "f64": 11}
RESIDENT = {"f32": (10, 12), "f64": (10, 11)}      # shapes resident_pass serves
COL_RANGES = ((0, 6), (7, 7), (8, 8))               # log2 n2 served by one column kernel
ROW_RANGES = ((0, 5), (6, 11), (12, 12))            # log2 n1 served by one row kernel
KEEP_DEFAULT = 0.02


def range_of(ranges, v):
    return next(i for i, (lo, hi) in enumerate(ranges) if lo <= v <= hi)


def split_of(l, prec, col_log2):
    """log2 n2 that the library's plan gives for nt = 2^l and a col_log2 option."""
    if col_log2 > 0 and l > 10:
        return max(min(col_log2, l // 2), l - MAX_LOG2_N1[prec])
    if l <= 12:
        return l // 2
    return max(6, l - MAX_LOG2_N1[prec])


def instances(l, nf, count):
    nt = 1 << l
    out = []
    for b in range(count):
        if nf == 3:
            w = W.config("sro_cw", nt=nt, nz=20, level=3.0, seed=1000 + b)
        else:
            w = W.config("degenerate_cw", nt=nt, nz=20, level=3.0, seed=1000 + b)
        out.append(dict(crystal=w["crystal"], cavity=w["cavity"], fields=w["fields"], pump_in=w["pump_in"]))
    return out


def time_candidate(insts, prec, col_log2, schedule, nz=20, warm=2, window_s=0.03, repeats=3):
    """ms per round trip: the best of `repeats` timings, each over enough round trips to
    last about window_s."""
    with B.Opo(insts, nz, precision=prec, col_log2=col_log2, schedule=schedule) as h:
        h.cavity_roundtrip(warm)
        t0 = time.perf_counter()
        h.cavity_roundtrip(2)
        reps = max(2, int(window_s / max((time.perf_counter() - t0) / 2, 1e-6)))
        best = None
        for _ in range(repeats):
            t0 = time.perf_counter()
            h.cavity_roundtrip(reps)
            dt = (time.perf_counter() - t0) / reps
            best = dt if best is None else min(best, dt)
    return best * 1e3


def tune(out, summary, precisions=("f32", "f64"), nfs=(3, 2)):
    rows, lines = [], []
    for prec in precisions:
        for nf in nfs:
            for l in range(10, MAX_LOG2[prec] + 1):
                for batched in (0, 1):
                    count = min(512, max(2, (1 << 22) >> l)) if batched else 1
                    if batched and count * (1 << l) * nf * (16 if prec == "f64" else 8) > (8 << 30):
                        continue
                    insts = instances(l, nf, count)
                    cands = []                      # (label, col_log2, resident, ms)
                    seen = set()
                    n2_default = split_of(l, prec, 0)
                    for cl in [0] + ([4, 5, 6, 7, 8] if l > 10 else []):
                        n2 = split_of(l, prec, cl)
                        if n2 in seen:
                            continue
                        # in a batch only splits served by the default's column and row
                        # kernels: any mix of batched shapes then keeps one column and one
                        # row kernel per half (the paired mixed launches)
                        if batched and (range_of(COL_RANGES, n2) != range_of(COL_RANGES, n2_default) or
                                        range_of(ROW_RANGES, l - n2) != range_of(ROW_RANGES, l - n2_default)):
                            continue
                        seen.add(n2)
                        ms = time_candidate(insts, prec, cl, "two_pass")
                        cands.append(("two-pass n2=2^%d" % n2, cl, 0, ms))
                    lo, hi = RESIDENT[prec]
                    if lo <= l <= hi:
                        ms = time_candidate(insts, prec, 0, "resident")
                        cands.append(("resident", 0, 1, ms))
                    default = cands[0]
                    best = min(cands, key=lambda c: c[3])
                    if best[3] > (1.0 - KEEP_DEFAULT) * default[3]:
                        best = default
                    rows.append((1 if prec == "f64" else 0, nf, l, batched, best[1], best[2]))
                    line = "%s nf=%d 2^%d %s x%d: " % (prec, nf, l, "batch" if batched else "alone", count) + \
                           ", ".join("%s %.3f ms" % (c[0], c[3]) for c in cands) + " -> " + best[0]
                    print(line, flush=True)
                    lines.append(line)
    with open(out, "w") as f:
        f.write("// schedule_table.inc -- {f64, nf, log2 nt, batched, {col_log2, resident}}, written by\n")
        f.write("// paper_2410_02532_amd/tune.py from round-trip times of every candidate on the device.\n")
        for r in rows:
            f.write("    {%d, %d, %d, %d, {%d, %d}},\n" % r)
    if summary:
        with open(summary, "w") as f:
            f.write("# Schedule tuning (ms per round trip of 20 steps per candidate)\n\n")
            f.write("Command: `python -m paper_2410_02532_amd.tune --out %s`\n\n" % os.path.basename(out))
            f.write("Each key times CW singly resonant oscillators of one shape, alone or as a batch of\n")
            f.write("about 2^22 points (batch candidates limited to the default's kernel size ranges),\n")
            f.write("best of three ~30 ms windows; the fastest candidate wins unless within 2 % of the\n")
            f.write("default.\n\n")
            for line in lines:
                f.write("- " + line + "\n")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(PKG, "csrc", "schedule_table.inc"))
    ap.add_argument("--summary", default=None)
    ap.add_argument("--precision", choices=("f32", "f64"), default=None)
    args = ap.parse_args()
    tune(args.out, args.summary, precisions=(args.precision,) if args.precision else ("f32", "f64"))


if __name__ == "__main__":
    main()
