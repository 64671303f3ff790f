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


def _bench_line(path, point, before):
    with open(path, "w") as f:
        f.write("[bench] noise\n")
        f.write(json.dumps({"operating_point": point, "kernels": {"delivery_launches_before_timed": before}}) + "\n")


def test_traffic_summary_scales_by_the_copy(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    copy = "void at::native::direct_copy_kernel_cuda(...)"
    d = "snn::k_deliver_tiled<512>"
    # the copy of 1 MiB reads 1024 KiB and the counter says 512: factor 2.  The stamped
    # pass made the run's last two delivery dispatches; the ones before are not counted
    _csv(str(tmp_path / "f" / "x" / "run_counter_collection.csv"), "FETCH_SIZE",
         [(copy, 512.0), (copy, 512.0), (copy, 512.0), (copy, 3.0), (d, 777.0), (d, 999.0), (d, 100.0),
          ("snn::k_update", 7.0), (d, 300.0)])
    _csv(str(tmp_path / "w" / "run_counter_collection.csv"), "WRITE_SIZE",
         [(copy, 1024.0), (copy, 1024.0), (copy, 1024.0), (copy, 0.0), (d, 66.0), (d, 55.0), (d, 10.0),
          (d, 10.0)])
    point = {"workload": bench.WORKLOAD, "settle_steps": 300, "warmup": 5, "steps": 20, "events": 123,
             "spikes": 4, "delivery": "tiled", "tiles": 87, "window": 15, "delivery_launches": 2}
    _bench_line(str(tmp_path / "a.json"), point, 1)
    _bench_line(str(tmp_path / "b.json"), point, 1)
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"),
                        [str(tmp_path / "a.json"), str(tmp_path / "b.json")], 1, "cmd")
    t = json.load(open(out))
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2)
    assert t["write_bytes_per_launch"] == pytest.approx(10.0 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2 + 10.0 * 1024)
    assert t["fetch_kib_per_dispatch"] == {"min": 100.0, "mean": 200.0, "max": 300.0}
    assert t["fetch_dispatches"] == 2 and t["write_dispatches"] == 2
    assert t["kernel_source_sha"] == bench.kernel_source_sha()
    assert bench.measured_traffic(point) == pytest.approx(t["bytes_per_launch"])
    # any other operating point gets no traffic figure
    for k, v in (("warmup", 6), ("events", 124), ("steps", 1000), ("tiles", 88)):
        assert bench.measured_traffic({**point, k: v}) is None
    # nor does another kernel source
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)
    assert bench.measured_traffic(point) is None


def test_traffic_summary_refuses_runs_at_different_points(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    point = {"workload": bench.WORKLOAD, "steps": 20, "events": 1}
    _bench_line(str(tmp_path / "a.json"), point, 1)
    _bench_line(str(tmp_path / "b.json"), {**point, "events": 2}, 1)
    with pytest.raises(SystemExit):
        bench.summarize_pmc(str(tmp_path), str(tmp_path), [str(tmp_path / "a.json"), str(tmp_path / "b.json")],
                            1, "cmd")


def test_launch_count_of_a_run():
    assert bench.launches_for(300, 15) == 20 and bench.launches_for(5, 15) == 1
    assert bench.launches_for(0, 15) == 0 and bench.launches_for(20, 15) == 2


def test_host_info_fields():
    h = bench.host_info()
    assert h["nproc"] >= 1 and set(h) == {"cpu_model", "nproc", "cpu_count", "ram_gib"}


def test_delivery_byte_model():
    """Per event: the target the delivery reads (2 B from the tiled delivery's 16-bit copy,
    4 B for the atomic delivery) plus a 4-byte weight when weights are stored per synapse;
    per dequeued spike: id + row pointers, plus the source weight in the Table I layout."""
    assert bench.delivery_bytes({"source_weights": 1, "target_bytes": 2}) == (2, 16)
    assert bench.delivery_bytes({"source_weights": 0, "target_bytes": 2}) == (6, 12)
    assert bench.delivery_bytes({"source_weights": 1, "target_bytes": 4}) == (4, 16)
    assert bench.delivery_bytes({"source_weights": 0, "target_bytes": 4}) == (8, 12)
