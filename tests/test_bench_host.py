"""Host-side logic of bench.py (no GPU): the one-GPU contract, the name of
the detection kernel a plan launches, and the traffic figures written from
counter runs."""
import csv
import json
import os
import subprocess
import sys

import pytest

import paper_1805_12258_amd as hs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_detection_kernel_names():
    """The kernel named in the bench line is the one the plan launches."""
    N = 1 << 21
    assert bench.detection_kernel(hs.Plan(85, N, 8))[0] == "k_fused<float,8,detect>"
    name, src = bench.detection_kernel(hs.Plan(85, N, 8, dtype="f16", input_scale=0.125), "f16")
    assert name == "k_walk<_Float16,8,8>" and any(s.endswith("hs_walk_f16_v8_g1.hip") for s in src)
    assert bench.detection_kernel(hs.Plan(85, N, 16))[0] == "k_walk<float,16,4>"
    assert bench.detection_kernel(hs.Plan(85, N, 8, mapping="fractional"))[0] == "k_frac<float,detect>"
    for _, src in (bench.detection_kernel(hs.Plan(85, N, 8)),
                   bench.detection_kernel(hs.Plan(85, N, 13, dtype="bf16", input_scale=0.125), "bf16")):
        assert all(os.path.exists(os.path.join(ROOT, s)) for s in src)


def _counter_csv(path, counter, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_summary(tmp_path, monkeypatch):
    """Medians of the detection kernel's dispatches, scaled by the plane
    copy's counters (small copies ignored), written with the source hash."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    plane_kib = 713031680 / 1024
    k = "void hsk::k_fused<float, 8, 0>(hsk::TileArgs, long)"
    other = "void hsk::k_fused<float, 8, 1>(hsk::TileArgs, long)"
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(k, 480000.0), (k, 490000.0), (k, 470000.0), (other, 1.0), (copy, plane_kib / 2), (copy, 3.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [(k, 2400.0), (k, 2500.0), (copy, plane_kib)])
    bench.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), {"schedule": 0}, ["c1", "c2"])
    d = json.load(open(tmp_path / "traffic.json"))
    assert d["kernel"] == "k_fused<float,8,detect>" and d["dispatches"] == [3, 2]
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    assert d["fetch_bytes"] == pytest.approx(480000.0 * 1024 * 2.0)
    assert d["write_bytes"] == pytest.approx(2450.0 * 1024)
    assert d["source_hash"] == bench.kernel_source_hash(bench.detection_kernel(hs.Plan(85, 1 << 21, 8))[1])
    assert os.path.exists(str(tmp_path / "traffic.md"))
    # the stored figures apply only to the same kernel and sources
    assert bench.stored_traffic("k_fused<float,8,detect>", bench.detection_kernel(hs.Plan(85, 1 << 21, 8))[1])
    assert bench.stored_traffic("k_walk<float,8,4>", []) is None
