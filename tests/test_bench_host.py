"""Host-side logic of bench.py (no GPU): the one-GPU guard and the HBM-traffic summary
built from rocprofv3 counter CSVs."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _csv(path, counter, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_summary_scales_by_the_copy(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    copy = "void at::native::direct_copy_kernel_cuda(...)"
    # the copy of 1 MiB reads 1024 KiB and the counter says 512: factor 2
    _csv(str(tmp_path / "f" / "x" / "run_counter_collection.csv"), "FETCH_SIZE",
         [(copy, 512.0), (copy, 512.0), (copy, 512.0), (copy, 3.0), ("snn::k_deliver_tiled<512>", 100.0),
          ("snn::k_deliver_tiled<512>", 300.0), ("snn::k_update", 7.0)])
    _csv(str(tmp_path / "w" / "run_counter_collection.csv"), "WRITE_SIZE",
         [(copy, 1024.0), (copy, 1024.0), (copy, 1024.0), (copy, 0.0), ("snn::k_deliver_tiled<512>", 10.0)])
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), 1, "cmd", skip=0)
    t = json.load(open(out))
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2)
    assert t["write_bytes_per_launch"] == pytest.approx(10.0 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2 + 10.0 * 1024)
    assert t["kernel_source_sha"] == bench.kernel_source_sha()
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.measured_traffic() == pytest.approx(t["bytes_per_launch"])


def test_delivery_byte_model():
    """Per event: the target the delivery reads (2 B from the tiled delivery's 16-bit copy,
    4 B for the atomic delivery) plus a 4-byte weight when weights are stored per synapse;
    per dequeued spike: id + row pointers, plus the source weight in the Table I layout."""
    assert bench.delivery_bytes({"source_weights": 1, "target_bytes": 2}) == (2, 16)
    assert bench.delivery_bytes({"source_weights": 0, "target_bytes": 2}) == (6, 12)
    assert bench.delivery_bytes({"source_weights": 1, "target_bytes": 4}) == (4, 16)
    assert bench.delivery_bytes({"source_weights": 0, "target_bytes": 4}) == (8, 12)
