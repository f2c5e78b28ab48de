"""Host logic of the HBM-traffic summary behind the benchmark's roofline line."""
import csv
import os

from paper_2410_02532_amd import traffic as T

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _run(tmp, name, counter, rows):
    d = os.path.join(tmp, name, "host")
    os.makedirs(d)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for disp, kern, val in rows:
            # a counter is reported per XCD: the summary adds the parts of one dispatch
            for part in (0.25, 0.75):
                w.writerow({"Dispatch_Id": disp, "Kernel_Name": kern, "Counter_Name": counter,
                            "Counter_Value": val * part})
    return os.path.join(tmp, name)


def test_summary_scales_by_the_copy_and_checks_the_sources(tmp_path):
    tmp = str(tmp_path)
    k = "void opo::mixed_pass<float, 0, 1>(opo::StepArgs<float>, opo::StepArgs<float>)"
    copy = "__amd_rocclr_copyBuffer"
    calib_kib = (256 << 20) / 1024.0
    # FETCH counts half the bytes of the copy, WRITE all of them
    fd = _run(tmp, "f", "FETCH_SIZE", [(1, copy, calib_kib / 2), (2, k, 1000.0), (3, k, 1200.0),
                                       (4, "void opo::column_pass<float, 0, 6>(x)", 9e9)])
    wd = _run(tmp, "w", "WRITE_SIZE", [(1, copy, calib_kib), (2, k, 500.0), (3, k, 700.0)])
    out = os.path.join(tmp, "s.md")
    m = T.summarize(fd, wd, "mixed_pass", out, "rocprofv3 --pmc FETCH_SIZE -- python bench.py")
    assert abs(m["fetch_scale"] - 2.0) < 1e-12 and abs(m["write_scale"] - 1.0) < 1e-12
    assert m["dispatches"] == (2, 2)
    assert abs(m["traffic_bytes"] - (1100.0 * 1024 * 2 + 600.0 * 1024)) < 1e-6
    assert T.load(out) == round(m["traffic_bytes"])
    # a summary taken on other kernel sources is not used
    text = open(out).read().replace(T.source_fingerprint(), "0" * 64)
    open(out, "w").write(text)
    assert T.load(out) is None
    assert T.load(os.path.join(tmp, "missing.md")) is None
