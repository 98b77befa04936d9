"""bench.py's counter summary (no GPU): per-launch HBM bytes from rocprofv3
counter CSVs, scaled by the device copy of the same run."""
import csv
import json
import os

import bench


def _counter_csv(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, value) in enumerate(rows):
            w.writerow([i, name, counter, value])


def test_summarize_counters(tmp_path, monkeypatch):
    traffic = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    copy = "__amd_rocclr_copyBuffer"
    bs = "void spk::k_bsweep_st<float, 64>(spk::ProbDev<float> const*)"
    pd = "void spk::k_prep<double, 32>(spk::ProbDev<double> const*)"
    # the 1 GiB copy reads FETCH_SIZE 512 Ki (factor 2) and WRITE_SIZE 1 Mi KiB (factor 1)
    _counter_csv(str(tmp_path / "f" / "run_counter_collection.csv"), "FETCH_SIZE",
                 [(copy, 3.0), (copy, 524288.0), (bs, 100.0), (bs, 300.0), (pd, 50.0)])
    _counter_csv(str(tmp_path / "w" / "run_counter_collection.csv"), "WRITE_SIZE",
                 [(copy, 1048576.0), (bs, 10.0), (pd, 4.0)])
    os.makedirs(tmp_path / "t")
    with open(tmp_path / "t" / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "AverageNs"])
        w.writerow([bs, 2, 80000.0])
    prof = {"copy_bytes": 1 << 30, "source_hash": "abc",
            "bytes_f32": {k: 1000.0 for k in bench.KERNELS}, "bytes_f64": {k: 2000.0 for k in bench.KERNELS}}
    (tmp_path / "p.json").write_text("log line\n" + json.dumps(prof) + "\n")
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "t"), str(tmp_path / "p.json"))
    out = json.loads(traffic.read_text())
    assert out["source_hash"] == "abc"
    assert abs(out["calibration"]["fetch_factor"] - 2.0) < 1e-9
    assert abs(out["calibration"]["write_factor"] - 1.0) < 1e-9
    b = out["kernels"]["k_bsweep<float>"]
    # mean FETCH_SIZE 200 KiB x 2 + WRITE_SIZE 10 KiB x 1
    assert b["fetch_bytes"] == 200 * 1024 * 2 and b["write_bytes"] == 10 * 1024
    assert b["algorithmic_bytes"] == 1000.0 and b["avg_us_trace"] == 80.0
    p = out["kernels"]["k_prep<double>"]
    assert p["bytes_per_launch"] == 50 * 1024 * 2 + 4 * 1024 and p["avg_us_trace"] is None
    assert "k_dual<float>" not in out["kernels"]


def test_batch_inputs_do_not_depend_on_the_pool():
    # members are seeded by their index: a process pool draws the same ones
    pooled, _, workers = bench.make_batch_inputs(6, workers=3)
    alone, _, one = bench.make_batch_inputs(6, workers=1)
    assert one == 1 and workers >= 1
    for a, b in zip(pooled, alone):
        for k, v in a.items():
            if hasattr(v, "tobytes"):
                assert v.tobytes() == b[k].tobytes(), k
            else:
                assert v == b[k], k
