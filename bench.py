"""Benchmark of the OPO split-step Fourier hot path on one MI355X.

A step is one cavity round trip of the whole hot path over one batch (nz
symmetrized SSFM steps with the fused RK4 half-steps, FFTs and dispersion
multiply, the round-trip boundary and the FP64 energy reduction, for every
instance of the batch in the same launches) replayed from a hipGraph.
The default workload is the batched sweep: 256 CW singly resonant OPOs with Nt
drawn from {2^12 .. 2^16}, pump 1-6x threshold, detuning +-0.5 rad, signal
R 0.90-0.99, Nz = 100, 500 round trips, complex64 fields with FP64 phase
arguments and energies, seeded synthetic inputs. Variants reported beside it:
one CW SRO at Nt = 2^14 (2000 round trips) in FP32 and in FP64.

Metric: field-point-steps per second = sum over instances of Nt * Nz * round
trips / time, with the inputs resident in HBM when the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2410_02532_amd import opo as B          # noqa: E402
from paper_2410_02532_amd import traffic as T      # noqa: E402
from paper_2410_02532_amd import workloads as W    # noqa: E402

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
# FP32 vector FMA issued one value per lane (the library is built without packed
# FP32 instructions): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
VALU_PEAK_TFLOPS = 78.6
VALU_PEAK_PACKED_TFLOPS = 157.3   # the same with packed (two-wide) FP32 FMA
BYTES_PER_FIELD = {"f32": 16, "f64": 32}   # read + write of one complex field


def nf_of(ins):
    return int(ins["crystal"].get("nf", 3))


def flops_per_unit(nt, nf=3):
    """Algorithmic flops of one field-point-step (all nf fields at one time point, one
    z-step): two RK4 half-steps (2 x 228 for three waves, two thirds of it for two), a
    forward and an inverse FFT of each field (nf x 2 x 5 log2 Nt) and the dispersion
    multiply (nf x 6)."""
    return 2 * 228 * nf / 3 + nf * 2 * 5 * np.log2(nt) + 6 * nf
METRIC = "field-point-steps/s (Nt*Nz*round trips/s)"


def instances_of(w):
    return w["instances"] if "instances" in w else [w]


def pt_steps_per_rt(w):
    return sum(ins["crystal"]["nt"] for ins in instances_of(w)) * w["nz"]


def timed_roundtrips(h, n_rt):
    """Device time (HIP events on the handle's stream) and wall time of n_rt round trips."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(h.stream)
    h.cavity_roundtrip(n_rt)
    e1.record(h.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def run_gpu(w, steps, warmup, precision, **kw):
    with B.from_workload(w, precision=precision, **kw) as h:
        if warmup:
            h.cavity_roundtrip(warmup)
        dev_s, wall_s = timed_roundtrips(h, steps)
    return dev_s, wall_s


def adaptive_run(w, repeats=3):
    """One adaptive-step propagation of the batch over the crystal length (timed after an
    untimed one that allocates the buffers; the fields are restored before each). value =
    accepted field-point-steps per second; every attempt runs three symmetrized steps."""
    import torch
    insts = instances_of(w)
    L = insts[0]["crystal"]["length_mm"]
    nts = np.array([i["crystal"]["nt"] for i in insts], dtype=np.float64)
    best = None
    with B.from_workload(w) as h:
        for r in range(repeats + 1):
            for b, ins in enumerate(insts):
                h.set_fields(ins["fields"], b)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(h.stream)
            acc, rej, _ = h.ssfm_propagate_adaptive(L, w["tol"], L / w["nz"])
            e1.record(h.stream)
            torch.cuda.synchronize()
            d = e0.elapsed_time(e1) / 1e3
            if r > 0 and (best is None or d < best[0]):
                best = (d, acc.copy(), rej.copy())
    d, acc, rej = best
    return {"value": float(np.sum(nts * acc) / d), "unit": "accepted field-point-steps/s",
            "ms": d * 1e3, "tol": w["tol"], "instances": len(insts),
            "accepted": [int(acc.min()), int(acc.max()), int(acc.sum())], "rejected": int(rej.sum()),
            "attempt_steps_per_s": float(3 * np.sum(nts * (acc + rej)) / d)}


def roofline(w, precision, n_rt):
    """Roofline of the dominant kernel from per-launch device times (HIP events around every
    launch, profile option).

    Each column, row or mixed launch carries out half of a z-step for the points it covers
    (a z-step is a column and a row pass of every instance), so its algorithmic work is half
    a field-point-step per covered point: 48/2 B and flops_per_unit/2 in FP32. The kernels
    issue more VALU work per byte than the FP32 ridge of the non-packed vector units, so the
    binding roofline is the ALU one; the HBM figure is reported beside it."""
    with B.from_workload(w, precision=precision, profile=True) as h:
        h.cavity_roundtrip(2)            # warm up
        before = h.kernel_times()
        h.cavity_roundtrip(n_rt)
        after = h.kernel_times()
    per = {k: (after[k][0] - before[k][0], after[k][1] - before[k][1]) for k in after}
    dom = max(("column_pass", "row_pass", "mixed_pass"), key=lambda k: per[k][0])
    ms, launches = per[dom]
    insts = instances_of(w)
    bytes_per_launch = sum(BYTES_PER_FIELD[precision] * nf_of(i) * i["crystal"]["nt"] for i in insts) / 2
    flops_per_launch = sum(i["crystal"]["nt"] * flops_per_unit(i["crystal"]["nt"], nf_of(i)) for i in insts) / 2
    avg_s = ms / 1e3 / launches
    tflops = flops_per_launch / avg_s / 1e12
    gbs = bytes_per_launch / avg_s / 1e9
    # HBM bytes per launch from the counter summary of this kernel and workload,
    # null unless it was taken on the current kernel sources
    traffic = T.load(os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.md" % (dom, w["name"], precision)))
    return {
        "bound": "alu", "kernel": dom, "achieved": round(tflops, 3), "peak": VALU_PEAK_TFLOPS,
        "unit": "TFLOP/s", "frac": round(tflops / VALU_PEAK_TFLOPS, 5), "traffic": traffic,
        "flops_per_launch": round(flops_per_launch), "avg_launch_us": round(avg_s * 1e6, 3),
        "frac_of_packed_peak": round(tflops / VALU_PEAK_PACKED_TFLOPS, 5),
        "hbm": {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 5), "bytes_per_launch": round(bytes_per_launch)},
        "kernel_ms": {k: round(v[0], 3) for k, v in per.items()},
        "launches": {k: v[1] for k, v in per.items()},
    }


def cpu_baseline(w, budget_s=12.0, max_rt=60):
    """The FP64 oracle, single-threaded, on a bounded sample of the same workload.

    The cost of a fixed-step round trip depends only on Nt, so the oracle runs
    round trips of the first instance of every size present until each size
    has had budget/len(sizes) seconds, and the batch rate is the workload's
    total points over the time those per-size costs add up to."""
    import oracle
    insts = instances_of(w)
    sizes = sorted({ins["crystal"]["nt"] for ins in insts})
    per_size = {}
    parts = []
    spent = 0.0
    for nt in sizes:
        ins = next(i for i in insts if i["crystal"]["nt"] == nt)
        a = ins["fields"]
        n_rt, t = 0, 0.0
        while n_rt < max_rt and t < budget_s / len(sizes):
            t0 = time.perf_counter()
            a, _ = oracle.roundtrips(ins["crystal"], ins["cavity"], a, ins["pump_in"], w["nz"], 1)
            t += time.perf_counter() - t0
            n_rt += 1
        per_size[nt] = t / n_rt
        spent += t
        parts.append("%d x %d RT" % (nt, n_rt))
    total_pts = sum(ins["crystal"]["nt"] for ins in insts) * w["nz"]
    total_t = sum(per_size[ins["crystal"]["nt"]] for ins in insts)
    return {"value": total_pts / total_t, "unit": "field-point-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": "%s: round trips from the seeded input of one instance per size (Nt x RT: "
                      "%s), Nz=%d, weighted by the workload's size mix; %.1f s on one host core"
                      % (w["name"], ", ".join(parts), w["nz"], spent)}


def copy_calibration(nbytes=256 << 20):
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copy calibration: %d bytes read, %d bytes written" % (nbytes, nbytes), file=sys.stderr)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed round trips")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batched_sweep")
    ap.add_argument("--precision", default="f32", choices=("f32", "f64"))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the single-instance FP32 and FP64 lines")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--adaptive-only", action="store_true",
                    help="only the adaptive-step variant (adaptive_pulsed), one JSON line")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU mode "
              "(batches shard by instance with no communication; see the design notes)",
              file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_calibration:
        copy_calibration()
    if args.adaptive_only:
        print(json.dumps(adaptive_run(W.config("adaptive_pulsed"))), flush=True)
        return 0

    w = W.config(args.workload, precision=args.precision) if args.workload == "sro_cw" else \
        W.config(args.workload)
    steps = args.steps if args.steps is not None else w["n_rt"]
    print("workload %s: %d instance(s), %d pt-steps per round trip, %d+%d round trips"
          % (args.workload, len(instances_of(w)), pt_steps_per_rt(w), args.warmup, steps),
          file=sys.stderr, flush=True)

    dev_s, wall_s = run_gpu(w, steps, args.warmup, args.precision)
    value = pt_steps_per_rt(w) * steps / dev_s
    print("timed: %.4f s device, %.4f s wall -> %.4g pt-steps/s" % (dev_s, wall_s, value),
          file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": value, "unit": "field-point-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": dev_s * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic (seeded noise and pump, workloads module)",
        "config": {"workload": args.workload, "instances": len(instances_of(w)),
                   "nt": sorted({ins["crystal"]["nt"] for ins in instances_of(w)}),
                   "nz": w["nz"], "round_trips": steps, "precision": args.precision,
                   "graph": True, "wall_s": round(wall_s, 4)},
    }
    if not args.no_roofline:
        line["roofline"] = roofline(w, args.precision, min(steps, 100))
        print("roofline: %s" % json.dumps(line["roofline"]), file=sys.stderr, flush=True)

    if not args.no_variants:
        var = {}
        for prec, n in (("f32", 2000), ("f64", 400)):
            ws = W.config("sro_cw", precision=prec)
            d, _ = run_gpu(ws, n, 10, prec)
            var["%s_single_sro_cw_2^14" % prec] = {"value": pt_steps_per_rt(ws) * n / d,
                                                  "round_trips": n, "ms_per_step": d * 1e3 / n}
            # the same with columns of 32 (col_log2 option): twice the column
            # workgroups, each with half the work, for an instance alone
            d, _ = run_gpu(ws, n, 10, prec, col_log2=5)
            var["%s_single_sro_cw_2^14_col32" % prec] = {"value": pt_steps_per_rt(ws) * n / d,
                                                        "round_trips": n, "ms_per_step": d * 1e3 / n}
        # the headline workload one instance at a time (a handle per instance, same
        # kernels): the batching gain on the same work
        if "instances" in w:
            n, tot_s, pts = 3, 0.0, 0
            for ins in w["instances"]:
                one = dict(ins, nz=w["nz"])
                d, _ = run_gpu(one, n, 1, args.precision)
                tot_s += d
                pts += ins["crystal"]["nt"] * w["nz"] * n
            var["%s_%s_one_at_a_time" % (args.precision, args.workload)] = {
                "value": pts / tot_s, "round_trips": n, "ms_per_step": tot_s * 1e3 / n}
        # the headline workload in FP64 (complex128 throughout)
        n = 50
        d, _ = run_gpu(w, n, 3, "f64")
        var["f64_%s" % args.workload] = {"value": pt_steps_per_rt(w) * n / d, "round_trips": n,
                                         "ms_per_step": d * 1e3 / n}
        # the synchronously pumped OPO at its largest grid, FP32 and FP64
        for prec in ("f32", "f64"):
            ws = W.config("sync_pumped", nt=1 << 18, precision=prec)
            n = 50
            d, _ = run_gpu(ws, n, 3, prec)
            var["%s_sync_pumped_2^18" % prec] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                                 "ms_per_step": d * 1e3 / n}
        # the large doubly resonant batch: 16 x 2^20, Nz 200, GDD and EOM
        ws = W.config("dro_large")
        n = 10
        d, _ = run_gpu(ws, n, 2, "f32")
        var["f32_dro_large_16x2^20"] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                        "ms_per_step": d * 1e3 / n}
        # the two-wave (degenerate) model over the same size mix
        ws = W.config("degenerate_sweep")
        n = 100
        d, _ = run_gpu(ws, n, 5, "f32")
        var["f32_degenerate_sweep"] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                       "ms_per_step": d * 1e3 / n, "instances": len(ws["instances"]),
                                       "fields": 2}
        # nanosecond regime: 10 ns pulses read one window per round trip, with the
        # per-round-trip record of the fields leaving the crystal
        ws = W.config("ns_pulsed")
        n = ws["n_rt"]
        with B.from_workload(ws, record_rt=n) as h:
            d, _ = timed_roundtrips(h, n)
        var["f32_ns_pulsed"] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                "ms_per_step": d * 1e3 / n, "instances": len(ws["instances"]),
                                "nt": ws["instances"][0]["crystal"]["nt"], "record": True}
        # adaptive step: 128 uneven-Nt single-pass amplifiers (gain-length 3-8, 2 ps pump,
        # mismatch spread), each choosing its own steps, tol 1e-5
        ws = W.config("adaptive_pulsed")
        var["f32_adaptive_pulsed"] = adaptive_run(ws)
        line["variants"] = var
        print("variants: %s" % json.dumps(var), file=sys.stderr, flush=True)

    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w)
        print("cpu baseline: %s" % json.dumps(line["cpu_baseline"]), file=sys.stderr, flush=True)

    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
