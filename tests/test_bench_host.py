"""Host-side logic of bench.py: the one-GPU guard, and turning profiler counter files
into HBM bytes per launch (no GPU work)."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_file(d, tag, rows):
    os.makedirs(os.path.join(d, tag))
    with open(os.path.join(d, tag, "pmc_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": v})


def test_write_traffic_scales_by_the_copy_calibration(tmp_path):
    d = str(tmp_path / "pmc")
    # the 1 GiB copy reads as half its size on FETCH_SIZE and exactly its size on WRITE_SIZE
    _counter_file(d, "fetch_copy", [("copyBuffer", 524288.0)] * 3)
    _counter_file(d, "write_copy", [("copyBuffer", 1048576.0)] * 3)
    _counter_file(d, "fetch_wl", [("void ghn::k_predict_dense<4, 0>(PredictArgs)", 1000.0),
                                  ("void ghn::k_predict_dense<4, 0>(PredictArgs)", 3000.0),
                                  ("void ghn::k_predict_group<4, 8, 1>(GroupArgs)", 50.0),
                                  ("some_other_kernel", 7.0)])
    _counter_file(d, "write_wl", [("void ghn::k_predict_dense<4, 0>(PredictArgs)", 10.0),
                                  ("void ghn::k_predict_dense<4, 0>(PredictArgs)", 30.0),
                                  ("void ghn::k_predict_group<4, 8, 1>(GroupArgs)", 5.0)])
    out_file = str(tmp_path / "traffic.json")
    out = bench.write_traffic(d, ["wl"], out_file)
    cal = out["copy_calibration"]
    assert cal["fetch_scale"] == 2.0 and cal["write_scale"] == 1.0
    t = out["wl/fp32"]
    assert t["kernel"] == "k_predict_dense" and t["dispatches"] == 2
    assert t["bytes_per_launch"] == (2000.0 * 2.0 + 20.0) * 1024.0
    assert t["source_sha256_16"] == bench.source_hash("k_predict_dense")
    g = out["wl/bf16"]
    assert g["bytes_per_launch"] == (50.0 * 2.0 + 5.0) * 1024.0
    assert json.load(open(out_file)) == json.loads(json.dumps(out))


def test_measured_traffic_only_for_the_configuration_it_was_taken_in(tmp_path, monkeypatch):
    """Counter bytes recorded at one cell width, ring schedule or grouping are not reported
    for a run in another configuration."""
    import argparse
    d = str(tmp_path / "pmc")
    _counter_file(d, "fetch_copy", [("copyBuffer", 524288.0)])
    _counter_file(d, "write_copy", [("copyBuffer", 1048576.0)])
    _counter_file(d, "fetch_wl", [("void ghn::k_predict_tree<8, 0>(PredictArgs)", 100.0),
                                  ("void ghn::k_predict_group<8, 8, 1>(GroupArgs)", 40.0)])
    _counter_file(d, "write_wl", [("void ghn::k_predict_tree<8, 0>(PredictArgs)", 1.0),
                                  ("void ghn::k_predict_group<8, 8, 1>(GroupArgs)", 2.0)])
    out_file = str(tmp_path / "traffic.json")
    args = argparse.Namespace(cell_width=0.5, ring_step=1, ring_grow=True, sort=True, group_levels=2, group_size=0,
                              tile_width=0)
    out = bench.write_traffic(d, ["wl"], out_file, args=args)
    assert out["wl/fp32"]["config"] == {"cell_width": 0.5, "ring_step": 1, "ring_grow": True, "sort": True}
    assert out["wl/bf16"]["config"] == {"cell_width": 0.5, "group_levels": 2, "group_size": 16, "tile_width": 64}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", out_file)
    run32 = {"cell_width": 0.5, "ring_step": 1, "ring_grow": True, "sort": True}
    run16 = {"cell_width": 0.5, "group_levels": 2, "group_size": 16, "tile_width": 64}
    assert bench.measured_traffic("wl", "fp32", run32, 0.25) == out["wl/fp32"]["bytes_per_launch"]
    assert bench.measured_traffic("wl", "bf16", run16, 0.25) == out["wl/bf16"]["bytes_per_launch"]
    assert bench.measured_traffic("wl", "fp32", dict(run32, cell_width=0.25), 0.25) is None
    assert bench.measured_traffic("wl", "fp32", dict(run32, ring_step=2), 0.25) is None
    assert bench.measured_traffic("wl", "fp32", dict(run32, sort=False), 0.25) is None
    assert bench.measured_traffic("wl", "bf16", dict(run16, group_levels=1), 0.25) is None
    assert bench.measured_traffic("wl", "bf16", dict(run16, tile_width=32), 0.25) is None
    # a width recorded as None is the workload's calibrated width
    args.cell_width = None
    out = bench.write_traffic(d, ["wl"], out_file, args=args)
    assert bench.measured_traffic("wl", "fp32", dict(run32, cell_width=0.25), 0.25) is not None
    assert bench.measured_traffic("wl", "fp32", run32, 0.25) is None
