"""Benchmark of the OPO split-step Fourier hot path on one MI355X.

A step is one cavity round trip of the whole hot path over one batch (nz
symmetrized SSFM steps with the fused RK4 half-steps, FFTs and dispersion
multiply, the round-trip boundary and the FP64 energy reduction, for every
instance of the batch in the same launches) replayed from a hipGraph.
The default workload is the batched sweep: 256 CW singly resonant OPOs with Nt
drawn from {2^12 .. 2^16}, pump 1-6x threshold, detuning +-0.5 rad, signal
R 0.90-0.99, Nz = 100, 500 round trips, complex64 fields with FP64 phase
arguments and energies, seeded synthetic inputs, the automatic schedule (the
2^12 instances run resident beside the two-pass launches of the others).
Variants reported beside it (FP64, one instance at a time, the single 2^14 SRO
with its automatic and its default split, the synchronously pumped 2^18 OPO,
the 16 x 2^20 DRO batch, the two-wave sweep, a sweep of 2^10..2^12 grids
resident and in two passes, the nanosecond regime and the adaptive step) each
carry their error against the FP64 oracle.

Metric: field-point-steps per second = sum over instances of Nt * Nz * round
trips / time, with the inputs resident in HBM when the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2410_02532_amd import opo as B          # noqa: E402
from paper_2410_02532_amd import traffic as T      # noqa: E402
from paper_2410_02532_amd import workloads as W    # noqa: E402

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
VALU_PEAK_TFLOPS = 157.3     # MI355X FP32 vector, published (two-wide packed FMA)
# the same units issuing one FP32 FMA per lane per cycle (this library is built
# without packed FP32 instructions): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
VALU_NONPACKED_TFLOPS = 78.6
BYTES_PER_FIELD = {"f32": 16, "f64": 32}   # read + write of one complex field
METRIC = "field-point-steps/s (Nt*Nz*round trips/s)"
GOLDEN = os.path.join(ROOT, "tests", "golden")
PAPER = {
    "claim": ">50x GPU over CPU for the full OPO simulation at vector size n = 2^14",
    "hardware": "NVIDIA GeForce GTX 1650 (CUDA, cuFFT) vs Intel Core i7-9700 @ 3.00 GHz (C, FFTW)",
    "precision": "FP32",
    "where": "abstract and Sec. 3.4",
    "comparable": False,
    "note": "the CPU side here is the plain FP64 oracle with its own radix-2 FFT, not FFTW",
}


def nf_of(ins):
    return int(ins["crystal"].get("nf", 3))


def flops_per_unit(nt, nf=3):
    """Algorithmic flops of one field-point-step (all nf fields at one time point, one
    z-step): two RK4 half-steps (2 x 228 for three waves, two thirds of it for two), a
    forward and an inverse FFT of each field (nf x 2 x 5 log2 Nt) and the dispersion
    multiply (nf x 6)."""
    return 2 * 228 * nf / 3 + nf * 2 * 5 * np.log2(nt) + 6 * nf


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


def run_gpu(w, steps, warmup, precision, keep=(), **kw):
    """Timed round trips; also returns the energy histories (from opo_init on) of the
    instances in keep."""
    with B.from_workload(w, precision=precision, **kw) as h:
        if warmup:
            h.cavity_roundtrip(warmup)
        dev_s, wall_s = timed_roundtrips(h, steps)
        hist = {i: h.energy_history(i) for i in keep}
    return dev_s, wall_s, hist


def plans(w, precision, **kw):
    """(log2 n1, log2 n2, resident) of every instance under the handle's schedule."""
    with B.from_workload(w, precision=precision, **kw) as h:
        return [h.plan(i) for i in range(len(instances_of(w)))]


# ------------------------------------------------------------------ errors --
# The oracle runs in worker processes while the GPU is being timed; each job
# regenerates its seeded input from the workloads module.

def _oracle_job(job):
    import oracle
    kind, name, over, idx, arg = job
    w = W.config(name, **over)
    ins = instances_of(w)[idx]
    cr, nz = ins["crystal"], w["nz"]
    if kind == "pass":
        return oracle.ssfm_pass(cr, ins["fields"], nz, cr["length_mm"] / nz)
    if kind == "rt":
        pump = np.asarray(ins["pump_in"])
        if pump.ndim == 2:
            return oracle.roundtrips_record(cr, ins["cavity"], ins["fields"], pump, nz, arg, record=False)[1]
        return oracle.roundtrips(cr, ins["cavity"], ins["fields"], ins["pump_in"], nz, arg)[1]
    if kind == "adaptive":
        L = cr["length_mm"]
        out, acc, rej = oracle.propagate_adaptive(cr, ins["fields"], L, w["tol"], L / nz)
        return out, acc, rej
    raise ValueError(kind)


class OracleJobs:
    """Oracle computations submitted up front and collected after the GPU timing."""

    def __init__(self, workers):
        self.ex = ProcessPoolExecutor(max_workers=workers) if workers > 0 else None
        self.fut = {}

    def submit(self, key, job):
        if self.ex is not None:
            self.fut[key] = self.ex.submit(_oracle_job, job)

    def get(self, key):
        f = self.fut.get(key)
        return None if f is None else f.result()

    def close(self):
        if self.ex is not None:
            self.ex.shutdown(wait=True)


def rel_l2_max(got, ref):
    """Largest relative L2 error over the fields (fields that are zero in the oracle are
    skipped)."""
    out = 0.0
    for g, r in zip(got, ref):
        n = np.linalg.norm(r)
        if n > 0:
            out = max(out, float(np.linalg.norm(g - r) / n))
    return out


def energy_errors(hist, ref, rows):
    """Largest relative error of the signal's recorded energy (the output signal power is
    a fixed multiple of it) and of every field's, over the given round trips."""
    h, r = np.asarray(hist)[rows], np.asarray(ref)[rows]
    rel = np.abs(h - r) / np.where(r > 0, r, 1.0)
    rel[r <= 0] = 0.0
    return float(rel[:, 1].max()), float(rel.max())


def golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def merge_long_run(parts):
    """The worst of several golden comparisons (None entries skipped), with the instances
    that had a stored run."""
    got = [x for x in parts if x is not None]
    if not got:
        return None
    return {"round_trips": min(x["last_rt"] for x in got), "instances_compared": len(got),
            "signal_power_rel": max(x["signal_power_rel"] for x in got),
            "energy_rel_all_fields": max(x["energy_rel_all_fields"] for x in got)}


def golden_error(hist, g):
    """Energy errors of a GPU history against a stored oracle run at its sampled round
    trips that the history covers."""
    if g is None:
        return None
    rts = [m for m in g["energy_rt"] if m < len(hist)]
    if not rts:
        return None
    ref = np.zeros((max(rts) + 1, 3))
    for m, e in zip(g["energy_rt"], g["energy"]):
        if m <= max(rts):
            ref[m] = e
    s, a = energy_errors(hist, ref, rts)
    return {"signal_power_rel": s, "energy_rel_all_fields": a, "last_rt": max(rts) + 1}


def gpu_pass(insts, nz, precision, **kw):
    """Fields of the given instances after one pass of nz steps of L/nz from their seeded
    inputs (one handle; an instance gives the same bits alone or in any batch)."""
    L = insts[0]["crystal"]["length_mm"]
    with B.Opo(insts, nz, precision=precision, **kw) as h:
        h.ssfm_propagate(nz, L / nz)
        return [h.get_fields(i) for i in range(len(insts))]


def picks_per_size(w, by_level=False):
    """One instance per Nt class: the first, or the one with the highest pump level."""
    out = []
    insts = instances_of(w)
    for nt in sorted({i["crystal"]["nt"] for i in insts}):
        cand = [b for b, i in enumerate(insts) if i["crystal"]["nt"] == nt]
        out.append(max(cand, key=lambda b: w["levels"][b]) if by_level else cand[0])
    return out


# ---------------------------------------------------------------- roofline --

def roofline(w, precision, n_rt, graph_rt_s=None):
    """Roofline of the dominant kernel from per-launch device times (HIP events around every
    launch on the handle's stream, profile option).

    Each column, row or mixed launch carries out half of a z-step for the points of the
    two-pass instances it covers (a z-step is a column and a row pass of every such
    instance), so its algorithmic work is half a field-point-step per covered point: 48/2 B
    (FP32) of HBM traffic and flops_per_unit/2. Instances that run resident are not covered
    by those launches. The line is priced against HBM (the algorithmic minimum of one read
    and one write of every field per z-step); the VALU figures stand beside it."""
    with B.from_workload(w, precision=precision, profile=True) as h:
        two_pass = [i for i in range(len(instances_of(w))) if not h.plan(i)[2]]
        h.cavity_roundtrip(2)            # warm up
        before = h.kernel_times()
        h.cavity_roundtrip(n_rt)
        after = h.kernel_times()
    per = {k: (after[k][0] - before[k][0], after[k][1] - before[k][1]) for k in after}
    dom = max(("column_pass", "row_pass", "mixed_pass", "resident_pass"), key=lambda k: per[k][0])
    if dom == "resident_pass":
        return resident_roofline(w, precision, per, two_pass, graph_rt_s)
    ms, launches = per[dom]
    insts = [instances_of(w)[i] for i in two_pass]
    bytes_per_launch = sum(BYTES_PER_FIELD[precision] * nf_of(i) * i["crystal"]["nt"] for i in insts) / 2
    flops_per_launch = sum(i["crystal"]["nt"] * flops_per_unit(i["crystal"]["nt"], nf_of(i)) for i in insts) / 2
    avg_s = ms / 1e3 / launches
    tflops = flops_per_launch / avg_s / 1e12
    gbs = bytes_per_launch / avg_s / 1e9
    # HBM bytes per launch from the counter summary of this kernel and workload,
    # null unless it was taken on the current kernel sources
    traffic = T.load(os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.md" % (dom, w["name"], precision)))
    return {
        "bound": "hbm", "kernel": dom, "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": traffic,
        "bytes_per_launch": round(bytes_per_launch), "avg_launch_us": round(avg_s * 1e6, 3),
        "valu": {"achieved": round(tflops, 3), "unit": "TFLOP/s", "flops_per_launch": round(flops_per_launch),
                 "peak": VALU_PEAK_TFLOPS, "frac": round(tflops / VALU_PEAK_TFLOPS, 5),
                 "peak_nonpacked": VALU_NONPACKED_TFLOPS,
                 "frac_nonpacked": round(tflops / VALU_NONPACKED_TFLOPS, 5)},
        "kernel_ms": {k: round(v[0], 3) for k, v in per.items()},
        "launches": {k: v[1] for k, v in per.items()},
        "instances_covered": len(insts),
    }


def resident_roofline(w, precision, per, two_pass, graph_rt_s):
    """Roofline of the resident launches when they dominate (all instances small). The
    resident launches of a round trip (one per shape) cover nz field-point-steps of every
    resident point and keep the fields on chip: their HBM traffic is one read and one write
    of the fields per round trip, far below the two-pass minimum, so the line is priced
    against the non-packed FP32 VALU peak (no packed FP32 in this build: 256 CUs x 4 SIMDs
    x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s). The time is the graph-timed round trip
    when given (the shapes run side by side there; the profile option serializes them),
    else the profile option's time per round trip."""
    ms, groups = per["resident_pass"]
    insts = [ins for i, ins in enumerate(instances_of(w)) if i not in set(two_pass)]
    flops = sum(i["crystal"]["nt"] * w["nz"] * flops_per_unit(i["crystal"]["nt"], nf_of(i)) for i in insts)
    hbm = sum(BYTES_PER_FIELD[precision] * nf_of(i) * i["crystal"]["nt"] for i in insts)
    avg_s = graph_rt_s if graph_rt_s else ms / 1e3 / groups
    tflops = flops / avg_s / 1e12
    return {
        "bound": "alu", "kernel": "resident_pass", "achieved": round(tflops, 3), "peak": VALU_NONPACKED_TFLOPS,
        "unit": "TFLOP/s", "frac": round(tflops / VALU_NONPACKED_TFLOPS, 5), "traffic": None,
        "flops_per_round_trip": round(flops), "avg_round_trip_us": round(avg_s * 1e6, 3),
        "serialized_round_trip_us": round(ms / groups * 1e3, 3),
        "frac_packed_peak": round(tflops / VALU_PEAK_TFLOPS, 5),
        "hbm_bytes_per_round_trip": round(hbm), "hbm_gbs": round(hbm / avg_s / 1e9, 2),
        "kernel_ms": {k: round(v[0], 3) for k, v in per.items()},
        "launches": {k: v[1] for k, v in per.items()},
        "instances_covered": len(insts),
    }


# ------------------------------------------------------------- CPU baseline --

def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, nproc


_CPU_W = None


def _cpu_init(name):
    global _CPU_W
    _CPU_W = W.config(name)


def _cpu_one_rt(i):
    import oracle
    ins = instances_of(_CPU_W)[i]
    oracle.roundtrips(ins["crystal"], ins["cavity"], ins["fields"], ins["pump_in"], _CPU_W["nz"], 1)
    return ins["crystal"]["nt"] * _CPU_W["nz"]


def cpu_baseline(w, budget_s=12.0, max_rt=60, pool_budget_s=10.0, max_workers=16):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload.

    Per core: round trips of the first instance of every size present until each size has
    had budget/len(sizes) seconds; the cost of a fixed-step round trip depends only on Nt,
    so the batch rate is the workload's total points over the time those per-size costs
    add up to. All cores: one round trip of each instance in workload order, spread over a
    process pool (at most max_workers processes), timed over about pool_budget_s."""
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
    model, nproc = host_info()
    out = {"value": total_pts / total_t, "unit": "field-point-steps/s", "cores": 1, "kind": "oracle",
           "host": model, "nproc": nproc,
           "sample": "%s: round trips from the seeded input of one instance per size (Nt x RT: "
                     "%s), Nz=%d, weighted by the workload's size mix; %.1f s on one host core"
                     % (w["name"], ", ".join(parts), w["nz"], spent)}
    workers = max(1, min(nproc or 1, max_workers))
    if "instances" in w and workers > 1:
        # instances in workload order until the estimated pool time reaches the budget
        jobs, est = [], 0.0
        for i, ins in enumerate(insts):
            jobs.append(i)
            est += per_size[ins["crystal"]["nt"]] / workers
            if est >= pool_budget_s:
                break
        with ProcessPoolExecutor(max_workers=workers, initializer=_cpu_init, initargs=(w["name"],)) as ex:
            list(ex.map(time.sleep, [0.5] * workers))   # every worker started and initialized
            t0 = time.perf_counter()
            pts = sum(ex.map(_cpu_one_rt, jobs))
            wall = time.perf_counter() - t0
        out["all_cores"] = {"value": pts / wall, "cores": workers, "instances": len(jobs),
                            "wall_s": round(wall, 2),
                            "sample": "one round trip of each of the first %d instances (workload order), "
                                      "one process per core" % len(jobs)}
    return out


def cpu_configs(budget_s=8.0):
    """The FP64 oracle per core on every configuration (bounded samples; the cost of a
    fixed step, and so of a round trip, does not change along a run): c0 a whole pass, c1
    and c2 round trips from their seeded inputs for about budget_s each, c3 the benchmark's
    own cpu_baseline sample (one core and all cores), c4 a partial pass of one instance
    (20 of its 200 steps; the boundary adds one step's worth of pointwise work per round
    trip)."""
    import oracle
    out = {}

    def rts(name, over, label):
        w = W.config(name, **over)
        a, n, t = w["fields"], 0, 0.0
        while n < 1 or (t < budget_s and n < 2000):
            t0 = time.perf_counter()
            a, _ = oracle.roundtrips(w["crystal"], w["cavity"], a, w["pump_in"], w["nz"], 1)
            t += time.perf_counter() - t0
            n += 1
        nt = w["crystal"]["nt"]
        out[label] = {"value": nt * w["nz"] * n / t, "unit": "field-point-steps/s", "cores": 1,
                      "sample": "%d round trip(s) of Nt = %d, Nz = %d from the seeded input, %.1f s"
                                % (n, nt, w["nz"], t)}

    w = W.config("single_pass")
    cr = w["crystal"]
    t0 = time.perf_counter()
    oracle.ssfm_pass(cr, w["fields"], w["nz"], cr["length_mm"] / w["nz"])
    t = time.perf_counter() - t0
    out["c0_single_pass_2^10"] = {"value": cr["nt"] * w["nz"] / t, "unit": "field-point-steps/s", "cores": 1,
                                  "sample": "the whole pass (Nz = %d), %.2f s" % (w["nz"], t)}
    rts("sro_cw", {}, "c1_sro_cw_2^14")
    for l in (16, 17, 18):
        rts("sync_pumped", dict(nt=1 << l), "c2_sync_pumped_2^%d" % l)
    out["c3_batched_sweep"] = cpu_baseline(W.config("batched_sweep"))
    w = W.config("dro_large")
    ins = w["instances"][0]
    cr = ins["crystal"]
    k = 20
    t0 = time.perf_counter()
    oracle.ssfm_pass(cr, ins["fields"], k, cr["length_mm"] / w["nz"])
    t = time.perf_counter() - t0
    out["c4_dro_large_2^20"] = {"value": cr["nt"] * k / t, "unit": "field-point-steps/s", "cores": 1,
                                "sample": "%d of the %d steps of one instance's pass, %.1f s" % (k, w["nz"], t)}
    model, nproc = host_info()
    return {"oracle_per_config": out, "kind": "oracle", "host": model, "nproc": nproc}


def copy_calibration(nbytes=256 << 20):
    """A plain device copy of known size, for scaling HBM counters."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copy calibration: %d bytes read, %d bytes written" % (nbytes, nbytes), file=sys.stderr)


def adaptive_run(w, repeats=3):
    """One adaptive-step propagation of the batch over the crystal length (timed after an
    untimed one that allocates the buffers; the fields are restored before each). value =
    accepted field-point-steps per second; every attempt runs three symmetrized steps.
    Also returns the fields of the last run."""
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
        fields = {i: h.get_fields(i) for i in range(len(insts))}
    d, acc, rej = best
    res = {"value": float(np.sum(nts * acc) / d), "unit": "accepted field-point-steps/s",
           "ms": d * 1e3, "tol": w["tol"], "instances": len(insts),
           "accepted": [int(acc.min()), int(acc.max()), int(acc.sum())], "rejected": int(rej.sum()),
           "attempt_steps_per_s": float(3 * np.sum(nts * (acc + rej)) / d)}
    return res, acc, rej, fields


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed round trips")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batched_sweep")
    ap.add_argument("--precision", default="f32", choices=("f32", "f64"))
    ap.add_argument("--count", type=int, default=None,
                    help="instances of a batched workload other than its default (same recipe)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the variants (FP64, single instance, other workloads)")
    ap.add_argument("--no-errors", action="store_true", help="skip the errors against the oracle")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="only the oracle's per-core rate on every configuration (no GPU), one JSON line")
    ap.add_argument("--adaptive-only", action="store_true",
                    help="only the adaptive-step variant (adaptive_pulsed), one JSON line")
    args = ap.parse_args()

    if args.cpu_configs:
        print(json.dumps(cpu_configs()), flush=True)
        return 0
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
        print(json.dumps(adaptive_run(W.config("adaptive_pulsed"))[0]), flush=True)
        return 0

    name = args.workload
    over = {} if args.count is None else dict(count=args.count)
    w = W.config(name, precision=args.precision, **over) if name == "sro_cw" else W.config(name, **over)
    steps = args.steps if args.steps is not None else w["n_rt"]
    errors = not args.no_errors
    variants = not args.no_variants
    _, nproc = host_info()
    jobs = OracleJobs(max(1, min(8, (nproc or 2) - 2)) if errors else 0)
    sweep = name == "batched_sweep" and not over     # the stored long runs are of the default batch
    head_picks = picks_per_size(w, by_level=True) if sweep else [0]
    if errors:
        for i in head_picks:
            jobs.submit(("head", i), ("pass", name, over, i, None))
        if variants:
            jobs.submit("sro_pass", ("pass", "sro_cw", {}, 0, None))
            jobs.submit("sync_pass", ("pass", "sync_pumped", dict(nt=1 << 18), 0, None))
            for l in (16, 17):
                jobs.submit(("sync_pass", l), ("pass", "sync_pumped", dict(nt=1 << l), 0, None))
            jobs.submit("sync_rt", ("rt", "sync_pumped", dict(nt=1 << 18), 0, 3))
            jobs.submit("dro_pass", ("pass", "dro_large", {}, 0, None))
            dsw = W.config("degenerate_sweep")
            for i in picks_per_size(dsw):
                jobs.submit(("deg_pass", i), ("pass", "degenerate_sweep", {}, i, None))
                jobs.submit(("deg_rt", i), ("rt", "degenerate_sweep", {}, i, 3))
            for i in picks_per_size(W.config("small_sweep"), by_level=True):
                jobs.submit(("small_pass", i), ("pass", "small_sweep", {}, i, None))
                jobs.submit(("small_rt", i), ("rt", "small_sweep", {}, i, 3))
            for i in range(3):
                jobs.submit(("ns_pass", i), ("pass", "ns_pulsed", {}, i, None))
                jobs.submit(("ns_rt", i), ("rt", "ns_pulsed", {}, i, 30))
            adw = W.config("adaptive_pulsed")
            order = sorted(range(len(adw["instances"])), key=lambda i: (adw["instances"][i]["crystal"]["nt"], i))
            ad_picks = order[:3]
            for i in ad_picks:
                jobs.submit(("ad", i), ("adaptive", "adaptive_pulsed", {}, i, None))

    print("workload %s: %d instance(s), %d pt-steps per round trip, %d+%d round trips"
          % (name, len(instances_of(w)), pt_steps_per_rt(w), args.warmup, steps),
          file=sys.stderr, flush=True)

    dev_s, wall_s, head_hist = run_gpu(w, steps, args.warmup, args.precision, keep=head_picks)
    value = pt_steps_per_rt(w) * steps / dev_s
    print("timed: %.4f s device, %.4f s wall -> %.4g pt-steps/s" % (dev_s, wall_s, value),
          file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": value, "unit": "field-point-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": dev_s * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic (seeded noise and pump, workloads module)",
        "config": {"workload": name, "instances": len(instances_of(w)),
                   "nt": sorted({ins["crystal"]["nt"] for ins in instances_of(w)}),
                   "nz": w["nz"], "round_trips": steps, "precision": args.precision,
                   "graph": True, "schedule": "auto",
                   "resident_instances": sum(p[2] for p in plans(w, args.precision)),
                   "wall_s": round(wall_s, 4)},
    }
    if not args.no_roofline:
        line["roofline"] = roofline(w, args.precision, min(steps, 100), graph_rt_s=dev_s / steps)
        if over:
            line["roofline"]["traffic"] = None   # the counter runs cover the default batch only
        print("roofline: %s" % json.dumps(line["roofline"]), file=sys.stderr, flush=True)

    var = {}
    if variants:
        for prec, n in (("f32", 2000), ("f64", 400)):
            ws = W.config("sro_cw", precision=prec)
            d, _, hs = run_gpu(ws, n, 10, prec, keep=(0,))
            var["%s_single_sro_cw_2^14" % prec] = {"value": pt_steps_per_rt(ws) * n / d,
                                                  "round_trips": n, "ms_per_step": d * 1e3 / n,
                                                  "_hist": hs[0]}
            var["%s_single_sro_cw_2^14" % prec]["split_log2_n1_n2"] = plans(ws, prec)[0][:2]
            # the same on the default split (columns of 64): the automatic schedule of an
            # instance alone takes columns of 32 (twice the column workgroups, each with
            # half the work)
            d, _, _ = run_gpu(ws, n, 10, prec, schedule="two_pass")
            var["%s_single_sro_cw_2^14_n2_64" % prec] = {"value": pt_steps_per_rt(ws) * n / d,
                                                        "round_trips": n, "ms_per_step": d * 1e3 / n}
        # the headline workload one instance at a time (a handle per instance, same
        # kernels): the batching gain on the same work
        if "instances" in w:
            n, tot_s, pts = 3, 0.0, 0
            for ins in w["instances"]:
                one = dict(ins, nz=w["nz"])
                d, _, _ = run_gpu(one, n, 1, args.precision)
                tot_s += d
                pts += ins["crystal"]["nt"] * w["nz"] * n
            var["%s_%s_one_at_a_time" % (args.precision, name)] = {
                "value": pts / tot_s, "round_trips": n, "ms_per_step": tot_s * 1e3 / n}
        # the headline workload in FP64 (complex128 throughout)
        n = 50
        d, _, hs = run_gpu(w, n, 3, "f64", keep=head_picks)
        var["f64_%s" % name] = {"value": pt_steps_per_rt(w) * n / d, "round_trips": n,
                                "ms_per_step": d * 1e3 / n, "_hist": hs}
        # the synchronously pumped OPO at its largest grid, FP32 and FP64
        for prec in ("f32", "f64"):
            ws = W.config("sync_pumped", nt=1 << 18, precision=prec)
            n = 50
            d, _, hs = run_gpu(ws, n, 3, prec, keep=(0,))
            var["%s_sync_pumped_2^18" % prec] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                                 "ms_per_step": d * 1e3 / n, "_hist": hs[0]}
        # its smaller grids (FP32)
        for l in (16, 17):
            ws = W.config("sync_pumped", nt=1 << l)
            n = 50
            d, _, _ = run_gpu(ws, n, 3, "f32")
            var["f32_sync_pumped_2^%d" % l] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                               "ms_per_step": d * 1e3 / n}
        # the large doubly resonant batch: 16 x 2^20, Nz 200, GDD and EOM
        ws = W.config("dro_large")
        n = 10
        d, _, hs = run_gpu(ws, n, 2, "f32", keep=(0, 8))
        var["f32_dro_large_16x2^20"] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                        "ms_per_step": d * 1e3 / n, "_hist": hs}
        # the two-wave (degenerate) model over the same size mix
        ws = W.config("degenerate_sweep")
        n = 100
        d, _, hs = run_gpu(ws, n, 5, "f32", keep=picks_per_size(ws))
        var["f32_degenerate_sweep"] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                       "ms_per_step": d * 1e3 / n, "instances": len(ws["instances"]),
                                       "fields": 2, "_hist": hs}
        # the paper's small grids: 256 instances of 2^10..2^12 points, where every instance
        # runs resident (one workgroup per instance for the whole round trip) under the
        # automatic schedule, against the same batch on two passes per z-step
        ws = W.config("small_sweep")
        n = 100
        d, _, hs = run_gpu(ws, n, 5, "f32", keep=picks_per_size(ws, by_level=True))
        d2, _, _ = run_gpu(ws, n, 5, "f32", schedule="two_pass")
        var["f32_small_sweep_2^10..2^12"] = {
            "value": pt_steps_per_rt(ws) * n / d, "round_trips": n, "ms_per_step": d * 1e3 / n,
            "instances": len(ws["instances"]), "resident_instances": sum(p[2] for p in plans(ws, "f32")),
            "two_pass_value": pt_steps_per_rt(ws) * n / d2, "_hist": hs}
        # nanosecond regime: 10 ns pulses read one window per round trip, with the
        # per-round-trip record of the fields leaving the crystal
        ws = W.config("ns_pulsed")
        n = ws["n_rt"]
        with B.from_workload(ws, record_rt=n) as h:
            d, _ = timed_roundtrips(h, n)
            hs = {i: h.energy_history(i) for i in range(3)}
        var["f32_ns_pulsed"] = {"value": pt_steps_per_rt(ws) * n / d, "round_trips": n,
                                "ms_per_step": d * 1e3 / n, "instances": len(ws["instances"]),
                                "nt": ws["instances"][0]["crystal"]["nt"], "record": True, "_hist": hs}
        # adaptive step: 128 uneven-Nt single-pass amplifiers (gain-length 3-8, 2 ps pump,
        # mismatch spread), each choosing its own steps, tol 1e-5
        ws = W.config("adaptive_pulsed")
        res, acc, rej, fields = adaptive_run(ws)
        res["_fields"], res["_acc"], res["_rej"] = fields, acc, rej
        var["f32_adaptive_pulsed"] = res
        print("variants timed", file=sys.stderr, flush=True)

    # ---- errors against the FP64 oracle (untimed; the oracle ran beside the GPU work)
    if errors:
        t0 = time.perf_counter()
        err = {}
        # per pass: the sampled instances after one pass from their seeded inputs
        insts = instances_of(w)
        got = gpu_pass([insts[i] for i in head_picks], w["nz"], args.precision)
        ref = [jobs.get(("head", i)) for i in head_picks]
        err["pass_rel_l2"] = max(rel_l2_max(g, r) for g, r in zip(got, ref))
        err["pass_instances"] = [int(i) for i in head_picks]
        if sweep:
            # long run: the highest-pump instance of every size class against stored oracle
            # runs of 500 round trips (a separate untimed run when the timed one was shorter)
            if min(len(v) for v in head_hist.values()) < 500:
                _, _, head_hist = run_gpu(w, 500, 0, args.precision, keep=head_picks)
            err["long_run"] = merge_long_run(
                [golden_error(head_hist[i], golden("batched_sweep_nt%d" % insts[i]["crystal"]["nt"]))
                 for i in head_picks])
        line["errors_vs_oracle"] = err
        if variants:
            sro_ref = jobs.get("sro_pass")
            for prec in ("f32", "f64"):
                ws = W.config("sro_cw", precision=prec)
                v = var["%s_single_sro_cw_2^14" % prec]
                v["pass_rel_l2"] = rel_l2_max(gpu_pass([ws], ws["nz"], prec)[0], sro_ref)
                v["long_run"] = golden_error(v.pop("_hist"), golden("sro_cw_2000rt"))
                var["%s_single_sro_cw_2^14_n2_64" % prec]["pass_rel_l2"] = rel_l2_max(
                    gpu_pass([ws], ws["nz"], prec, schedule="two_pass")[0], sro_ref)
            v = var["f64_%s" % name]
            hs = v.pop("_hist")
            v["pass_rel_l2"] = max(rel_l2_max(g, r) for g, r in zip(
                gpu_pass([insts[i] for i in head_picks], w["nz"], "f64"), ref))
            if sweep:
                v["long_run"] = merge_long_run(
                    [golden_error(hs[i], golden("batched_sweep_nt%d" % insts[i]["crystal"]["nt"]))
                     for i in head_picks])
            sync_rt = jobs.get("sync_rt")
            for prec in ("f32", "f64"):
                ws = W.config("sync_pumped", nt=1 << 18, precision=prec)
                v = var["%s_sync_pumped_2^18" % prec]
                v["pass_rel_l2"] = rel_l2_max(gpu_pass([ws], ws["nz"], prec)[0], jobs.get("sync_pass"))
                s, a = energy_errors(v.pop("_hist"), sync_rt, [0, 1, 2])
                v["short_run"] = {"round_trips": 3, "signal_power_rel": s, "energy_rel_all_fields": a}
            for l in (16, 17):
                ws = W.config("sync_pumped", nt=1 << l)
                var["f32_sync_pumped_2^%d" % l]["pass_rel_l2"] = rel_l2_max(
                    gpu_pass([ws], ws["nz"], "f32")[0], jobs.get(("sync_pass", l)))
            ws = W.config("dro_large")
            v = var["f32_dro_large_16x2^20"]
            v["pass_rel_l2"] = rel_l2_max(gpu_pass([ws["instances"][0]], ws["nz"], "f32")[0], jobs.get("dro_pass"))
            hs = v.pop("_hist")
            v["short_run"] = merge_long_run([golden_error(hs[0], golden("dro_large_inst0")),
                                             golden_error(hs[8], golden("dro_large_inst8"))])
            ws = W.config("degenerate_sweep")
            v = var["f32_degenerate_sweep"]
            hs = v.pop("_hist")
            dp = picks_per_size(ws)
            gotd = gpu_pass([ws["instances"][i] for i in dp], ws["nz"], "f32")
            v["pass_rel_l2"] = max(rel_l2_max(g, jobs.get(("deg_pass", i))) for g, i in zip(gotd, dp))
            ee = [energy_errors(hs[i], jobs.get(("deg_rt", i)), [0, 1, 2]) for i in dp]
            v["short_run"] = {"round_trips": 3, "signal_power_rel": max(x[0] for x in ee),
                              "energy_rel_all_fields": max(x[1] for x in ee)}
            ws = W.config("small_sweep")
            v = var["f32_small_sweep_2^10..2^12"]
            hs = v.pop("_hist")
            sp = picks_per_size(ws, by_level=True)
            gots = gpu_pass([ws["instances"][i] for i in sp], ws["nz"], "f32")   # a batch: resident
            v["pass_rel_l2"] = max(rel_l2_max(g, jobs.get(("small_pass", i))) for g, i in zip(gots, sp))
            ee = [energy_errors(hs[i], jobs.get(("small_rt", i)), [0, 1, 2]) for i in sp]
            v["short_run"] = {"round_trips": 3, "signal_power_rel": max(x[0] for x in ee),
                              "energy_rel_all_fields": max(x[1] for x in ee)}
            ws = W.config("ns_pulsed")
            v = var["f32_ns_pulsed"]
            hs = v.pop("_hist")
            gotn = gpu_pass(ws["instances"], ws["nz"], "f32")
            v["pass_rel_l2"] = max(rel_l2_max(gotn[i], jobs.get(("ns_pass", i))) for i in range(3))
            ee = [energy_errors(hs[i], jobs.get(("ns_rt", i)), list(range(30))) for i in range(3)]
            v["short_run"] = {"round_trips": 30, "signal_power_rel": max(x[0] for x in ee),
                              "energy_rel_all_fields": max(x[1] for x in ee)}
            v = var["f32_adaptive_pulsed"]
            fields, acc, rej = v.pop("_fields"), v.pop("_acc"), v.pop("_rej")
            worst, same = 0.0, True
            for i in ad_picks:
                out, ra, rr = jobs.get(("ad", i))
                worst = max(worst, rel_l2_max(fields[i], out))
                same = same and (int(acc[i]), int(rej[i])) == (ra, rr)
            v["rel_l2_vs_oracle"] = worst
            v["same_steps_as_oracle"] = same
            v["checked_instances"] = [int(i) for i in ad_picks]
        print("errors vs oracle: %.1f s after the GPU work" % (time.perf_counter() - t0), file=sys.stderr,
              flush=True)
    jobs.close()
    for name_v, v in var.items():
        for k in [k for k in v if k.startswith("_")]:
            del v[k]
        # whole-run rate against the HBM roofline at the algorithmic bytes of one read and
        # one write of every field per z-step (resident instances can exceed 1)
        if v.get("unit", "field-point-steps/s") == "field-point-steps/s":
            nf = 2 if "degenerate" in name_v else 3
            bpu = nf * 2 * (16 if name_v.startswith("f64") else 8)
            v["hbm_frac_algorithmic"] = round(v["value"] * bpu / (HBM_PEAK_GBS * 1e9), 5)
    if var:
        line["variants"] = var
        print("variants: %s" % json.dumps(var), file=sys.stderr, flush=True)

    if not args.no_cpu:
        cpu = cpu_baseline(w)
        line["cpu_baseline"] = cpu
        print("cpu baseline: %s" % json.dumps(cpu), file=sys.stderr, flush=True)
        line["paper_context"] = dict(PAPER, this_gpu_over_oracle_one_core=round(value / cpu["value"], 1))
        if "all_cores" in cpu:
            line["paper_context"]["this_gpu_over_oracle_all_cores"] = round(value / cpu["all_cores"]["value"], 1)
    else:
        line["paper_context"] = PAPER

    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
