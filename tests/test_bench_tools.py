"""The measurement's conversions of profiler output, on small synthetic
inputs whose answers are known by construction: the HBM byte scaling by the
calibration copy, and the busy / idle split of a kernel trace inside the
timed window."""
import csv
import json

import numpy as np
import pytest

import bench


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


GRAD = "void pncg::k_grad<float, 0, false, 0, true, 448>(pncg::Args<float>, int, int, double*, double*)"
DIR = "void pncg::k_dir<float, false, 0, 384>(pncg::Args<float>, int)"
COPY = "__amd_rocclr_copyBuffer"


def test_traffic_scaled_by_the_calibration_copy(tmp_path):
    # the copy of CALIB_BYTES reads as half of them on FETCH_SIZE and all of
    # them on WRITE_SIZE (KiB): the kernels' figures scale by 2 and 1
    kib = bench.CALIB_BYTES / 1024.0
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    fetch_rows = [[COPY, "FETCH_SIZE", kib / 2]] * 3 + [[COPY, "FETCH_SIZE", 1.0]] + \
        [[GRAD, "FETCH_SIZE", v] for v in (100.0, 7000.0, 7000.0, 7100.0, 6900.0)] + \
        [[DIR, "FETCH_SIZE", 4000.0]]
    write_rows = [[COPY, "WRITE_SIZE", kib]] * 3 + \
        [[GRAD, "WRITE_SIZE", v] for v in (10.0, 900.0, 910.0)] + [[DIR, "WRITE_SIZE", 200.0]]
    f, w, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "traffic.json"
    _write_csv(f, hdr, fetch_rows)
    _write_csv(w, hdr, write_rows)
    res = bench.traffic_from_csv(str(f), str(w), str(out))
    assert res["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert res["calibration"]["write_scale"] == pytest.approx(1.0)
    # medians: grad fetch 7000 KiB, grad write 900 KiB (the no-op dispatch is an outlier)
    assert res["detail"]["grad"]["fetch_bytes"] == round(7000 * 1024 * 2.0)
    assert res["detail"]["grad"]["write_bytes"] == round(900 * 1024 * 1.0)
    assert res["pile"]["grad"] == round(7000 * 1024 * 2.0 + 900 * 1024)
    assert res["pile"]["dir"] == round(4000 * 1024 * 2.0 + 200 * 1024)
    assert res["detail"]["grad"]["dispatches"] == [5, 3]
    assert json.load(open(out))["pile"] == res["pile"]


def test_trace_gaps_inside_the_window(tmp_path):
    # kernels (start, end) in ns; the window (monotonic clock) holds the
    # middle four, the other clock's window holds none
    ks = [(0, 50, COPY), (1000, 3000, GRAD), (3500, 4500, DIR), (5000, 7000, GRAD), (9000, 10000, DIR),
          (20000, 21000, COPY)]
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    tr = tmp_path / "trace.csv"
    _write_csv(tr, hdr, [[n, s, e] for s, e, n in ks])
    win = {"start": {"monotonic": 500, "clock_boottime": 50000}, "end": {"monotonic": 15000, "clock_boottime": 60000},
           "frames": 2, "iters": 2}
    wj = tmp_path / "window.json"
    wj.write_text(json.dumps(win))
    g = bench.trace_gaps(str(tr), str(wj))
    assert g["clock"] == "monotonic"
    assert g["kernels"] == 4 and g["grad_launches"] == 2
    span, busy = 10000 - 1000, 2000 + 1000 + 2000 + 1000
    assert g["span_us"] == pytest.approx(span / 1e3)
    assert g["busy_us"] == pytest.approx(busy / 1e3)
    assert g["idle_frac"] == pytest.approx((span - busy) / span, abs=1e-4)
    assert g["idle_us_per_frame"] == pytest.approx((span - busy) / 1e3 / 2, abs=0.05)
    gaps = {t["between"]: t for t in g["top_gaps"]}
    # gaps: grad->dir 500, dir->grad 500, grad->dir 2000
    gd = gaps["k_grad<float, 0, false, 0, true, 448> -> k_dir<float, false, 0, 384>"]
    assert gd["count"] == 2 and gd["total_us"] == pytest.approx(2.5)
    assert np.isclose(sum(t["total_us"] for t in g["top_gaps"]), (span - busy) / 1e3)
