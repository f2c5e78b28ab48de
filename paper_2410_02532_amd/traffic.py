"""HBM traffic per launch from rocprofv3 counter runs, for the benchmark's roofline line.

Two `rocprofv3 --pmc` runs of the benchmark with `--copy-calibration`, one
collecting FETCH_SIZE and one WRITE_SIZE (KiB per dispatch), give the bytes a
kernel moves through HBM. Each counter is scaled by what it reads for the
calibration copy, a plain device-to-device copy of 256 MiB (read once,
written once), so the figure is in bytes the copy would call one read and one
write.

`summarize` writes a short text summary (profiles/) holding the per-launch
figure and a fingerprint of the kernel sources; `load` returns that figure
only while the sources still have that fingerprint, else None.

Usage (after the two pmc runs):
  python -m paper_2410_02532_amd.traffic FETCH_DIR WRITE_DIR KERNEL OUT.md "COMMAND"
"""
import csv
import glob
import hashlib
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CALIB_BYTES = 256 << 20


def source_fingerprint():
    """SHA-256 over the HIP sources and headers the library is built from."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(PKG, "csrc", "*"))) + [os.path.join(ROOT, "include", "opo.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _per_dispatch(run_dir, counter):
    """{kernel name: [value per dispatch]} for one counter from a rocprofv3 csv run."""
    out = {}
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            acc = {}
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
                acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
        for (name, _), v in acc.items():
            out.setdefault(name, []).append(v)
    return out


def _short(name):
    return name.split("(")[0].replace("void ", "").strip()


def _copy_kernel(d):
    cands = [k for k in d if "copy" in k.lower()]
    if not cands:
        raise SystemExit("no copy kernel in the counter run (was --copy-calibration passed?)")
    # the calibration copy is the largest copy dispatch
    return max(cands, key=lambda k: max(d[k]))


def measure(fetch_dir, write_dir, kernel):
    fd = _per_dispatch(fetch_dir, "FETCH_SIZE")
    wd = _per_dispatch(write_dir, "WRITE_SIZE")
    ck_f, ck_w = _copy_kernel(fd), _copy_kernel(wd)
    copy_f, copy_w = max(fd[ck_f]), max(wd[ck_w])
    f_scale = CALIB_BYTES / (copy_f * 1024.0)
    w_scale = CALIB_BYTES / (copy_w * 1024.0)
    kf = [k for k in fd if _short(k).split("<")[0].endswith(kernel)]
    kw = [k for k in wd if _short(k).split("<")[0].endswith(kernel)]
    if not kf or not kw:
        raise SystemExit("kernel %s not in the counter runs" % kernel)
    fv = [v for k in kf for v in fd[k]]
    wv = [v for k in kw for v in wd[k]]
    fetch_b = sum(fv) / len(fv) * 1024.0 * f_scale
    write_b = sum(wv) / len(wv) * 1024.0 * w_scale
    return {
        "kernel": kernel, "instantiations": sorted({_short(k) for k in kf}),
        "dispatches": (len(fv), len(wv)),
        "fetch_kib": sum(fv) / len(fv), "write_kib": sum(wv) / len(wv),
        "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "fetch_bytes": fetch_b, "write_bytes": write_b, "traffic_bytes": fetch_b + write_b,
    }


def summarize(fetch_dir, write_dir, kernel, out_md, command):
    m = measure(fetch_dir, write_dir, kernel)
    lines = [
        "# HBM traffic of `%s`" % kernel, "",
        "Counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own",
        "`rocprofv3 --pmc` run, scaled by the same counter over a plain 256 MiB",
        "device copy (read once, written once) in the same run.", "",
        "Commands (FETCH_SIZE run, then the same with WRITE_SIZE):", "", "```", command, "```", "",
        "| | FETCH_SIZE | WRITE_SIZE |", "|---|---|---|",
        "| `%s`, mean per dispatch (KiB) | %.1f | %.1f |" % (kernel, m["fetch_kib"], m["write_kib"]),
        "| dispatches | %d | %d |" % m["dispatches"],
        "| 256 MiB copy (KiB) | %.1f | %.1f |" % (m["copy_fetch_kib"], m["copy_write_kib"]),
        "| scale (bytes per counted KiB / 1024) | %.4f | %.4f |" % (m["fetch_scale"], m["write_scale"]),
        "| bytes per launch | %.4g | %.4g |" % (m["fetch_bytes"], m["write_bytes"]), "",
        "Instantiations: %s" % ", ".join("`%s`" % s for s in m["instantiations"]), "",
        "traffic_bytes_per_launch: %d" % round(m["traffic_bytes"]),
        "kernel_sources_sha256: %s" % source_fingerprint(), "",
    ]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    return m


def load(summary_md):
    """Traffic bytes per launch from a summary, or None if it is missing or the kernel
    sources changed since the counters were taken."""
    try:
        with open(summary_md) as f:
            text = f.read()
    except OSError:
        return None
    tb = re.search(r"^traffic_bytes_per_launch: (\d+)$", text, re.M)
    fp = re.search(r"^kernel_sources_sha256: ([0-9a-f]{64})$", text, re.M)
    if not tb or not fp or fp.group(1) != source_fingerprint():
        return None
    return int(tb.group(1))


if __name__ == "__main__":
    if len(sys.argv) != 6:
        print(__doc__, file=sys.stderr)
        sys.exit(2)
    res = summarize(*sys.argv[1:6])
    print("traffic %.4g B per launch (fetch %.4g, write %.4g)"
          % (res["traffic_bytes"], res["fetch_bytes"], res["write_bytes"]))
