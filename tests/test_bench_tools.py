"""Host logic of the measurement tooling in bench.py (CPU): the traffic summary
picks the timed applies out of a counter run that also holds the schedule
tuning, and scales each counter by the plain copy of known size."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for did, name, val in rows:
            w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val})


def test_summarize_traffic_takes_the_timed_applies(tmp_path):
    steps, D = 3, 1000
    tune = [(1, "void ed::k_rt<float, float, 2, 512>(x)", 999.0), (2, "void ed::k_gtile<float, float, 4, 256>(x)", 999.0),
            (3, "void ed::k_cs<float, float, 512>(x)", 999.0), (4, "void ed::k_upb<float, float, 2, 128>(x)", 999.0)]
    # the timed schedule: two kernels per apply (a row pass and a band pass)
    timed = []
    for i in range(steps):
        timed.append((10 + 2 * i, "void ed::k_cs<float, float, 512>(x)", 10.0))
        timed.append((11 + 2 * i, "void ed::k_upb<float, float, 2, 128>(x)", 6.0))
    copies = [(30 + i, "__amd_rocclr_copyBuffer", 2.0) for i in range(steps)]   # KiB per copy as read
    fetch, write = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    _counter_csv(fetch, "FETCH_SIZE", tune + timed + copies)
    _counter_csv(write, "WRITE_SIZE", tune + timed + copies)
    info = str(tmp_path / "pass.log")
    with open(info, "w") as f:
        f.write("[bench] pmc-pass\n")
        f.write(json.dumps({"workload": "ns15", "D": D, "order": "grouped", "schedules": ["csx_demo"], "steps": steps,
                            "copy_bytes_each_way": 4 * D}) + "\n")
    out = bench.summarize_traffic(fetch, write, info, "demo")["demo"]
    # the copy moves 4 D = 4000 B each way but the counter read 2 KiB: factor 4000 / 2048
    factor = 4000.0 / 2048.0
    assert abs(out["fetch_factor"] - factor) < 1e-12
    assert abs(out["fetch_bytes"] - 16.0 * 1024.0 * factor) < 1e-6      # (10 + 6) KiB per apply
    assert abs(out["bytes_per_launch"] - 2 * 16.0 * 1024.0 * factor) < 1e-6
    assert sorted(out["kernels"]) == sorted(["void ed::k_cs<float, float, 512>(x)",
                                             "void ed::k_upb<float, float, 2, 128>(x)"])
    assert out["schedule"] == "csx_demo" and out["algorithmic_bytes"] == 8 * D


def test_summarize_stats_orders_by_total_time(tmp_path):
    path = str(tmp_path / "stats.csv")
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs"])
        w.writeheader()
        w.writerow({"Name": "a", "Calls": 10, "AverageNs": 100.0})
        w.writerow({"Name": "b", "Calls": 1, "AverageNs": 5000.0})
        w.writerow({"Name": "c", "Calls": 100, "AverageNs": 1.0})
    assert [n for n, _, _ in bench.summarize_stats(path)] == ["b", "a", "c"]


def test_step_roofline():
    r = bench.step_roofline({"traffic": 8e12, "iters": 100}, 2.0)
    assert r["GBps"] == 4000.0 and r["frac"] == 0.5 and r["ms_per_step"] == 20.0
