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
