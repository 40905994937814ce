"""Host-side logic of the measurement tools (no GPU): the traffic records' schedule keys
and the HBM-byte arithmetic of bench_traffic.py on synthetic counter files."""

import csv
import json
import os

import pytest

import bench_traffic as traffic


def test_schedule_keys():
    # default double plan at N = 2^20: split 0, two rows per pass-B tile, XCD order,
    # four-column pass-A/C tiles
    assert traffic.schedule_key(0, 0, 1, 1) == {"split": 0, "rows_b": 2, "xcd": 1, "cols_ac": 4}
    assert traffic.schedule_key(0, 2, 1, 0) == {"split": 0, "rows_b": 2, "xcd": 1, "cols_ac": 8}
    assert traffic.schedule_key(0, 4, 0, 0)["rows_b"] == 4
    # with split 1, L1 = 2^11 at N = 2^20: the narrow knob does not apply
    assert traffic.schedule_key(1, 2, 1, 1)["cols_ac"] == 8


def _write_counters(d, counter, values):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for name, vals in values.items():
            for v in vals:
                wr.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_arithmetic(tmp_path, monkeypatch):
    """Per-dispatch means of the three passes, scaled by what each counter reads for a
    1 GiB copy, summed; the record is keyed by the environment's schedule."""
    kA = "void birk::fast::k_fastA2<double, 10, 2>(...)"
    kB = "void birk::fast::k_fastB2<double, 0, 11, 2>(...)"
    kC = "void birk::fast::k_fastC2<double, 0, 10, 2>(...)"
    kBT = "void birk::fast::k_fastB2<double, 1, 11, 2>(...)"   # transposed: not counted
    copy = "__amd_rocclr_copyBuffer"
    d = tmp_path
    _write_counters(str(d / "f"), "FETCH_SIZE", {kA: [100, 300], kB: [400], kC: [50], kBT: [9999]})
    _write_counters(str(d / "w"), "WRITE_SIZE", {kA: [10], kB: [20], kC: [30, 50]})
    _write_counters(str(d / "cf"), "FETCH_SIZE", {copy: [524288]})      # 1 GiB / 2048
    _write_counters(str(d / "cw"), "WRITE_SIZE", {copy: [1048576]})     # 1 GiB / 1024
    out = d / "t.json"
    monkeypatch.setenv("BIRK_FAST_NARROW", "1")
    monkeypatch.setattr("sys.argv", ["traffic", str(d / "f"), str(d / "w"), str(d / "cf"), str(d / "cw"), str(out)])
    traffic.main()
    rec = json.load(open(out))["records"][0]
    assert rec["schedule"] == {"split": 0, "rows_b": 2, "xcd": 1, "cols_ac": 4}
    expect = (200 + 400 + 50) * 2048 + (10 + 20 + 40) * 1024
    assert rec["bytes_per_product"] == pytest.approx(expect)
