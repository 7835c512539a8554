"""Host-side checks of bench.py's bookkeeping: the one-GPU guard, and the
counter traffic it attaches to a roofline (only from counters taken on the
same kernel sources and the same workload).  No device work is issued."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _traffic_file(tmp_path, hash_, workloads):
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({"kernels_hash": hash_, "fetch_scale": 2.0, "write_scale": 1.0, "workloads": workloads}))
    return str(p)


def test_traffic_only_for_matching_sources_and_workload(bench, tmp_path, monkeypatch):
    wl = {"campaign": {"per_launch_bytes": {"k_pairs_sp": 1000}},
          "single_pulse_10um": {"per_launch_bytes": {"k_pairs_sp": 500}}}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, bench.kernels_hash(), wl))
    assert bench.measured_traffic("campaign", "k_pairs_sp") == 1000
    assert bench.measured_traffic("single_pulse_10um", "k_pairs_sp") == 500
    assert bench.measured_traffic("campaign", "k_bin") is None
    assert bench.measured_traffic("other", "k_pairs_sp") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, "0" * 16, wl))
    assert bench.measured_traffic("campaign", "k_pairs_sp") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.measured_traffic("campaign", "k_pairs_sp") is None


def test_counter_rate_from_mean_launch_time(bench, tmp_path, monkeypatch):
    wl = {"campaign": {"per_launch_bytes": {"k_scatter": 8_000_000}}}
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _traffic_file(tmp_path, bench.kernels_hash(), wl))
    r = bench.add_traffic({"kernel": "k_scatter", "avg_launch_us": 2.0}, "campaign")
    # 8 MB in 2 us = 4 TB/s, half of the 8 TB/s peak
    assert r["traffic"] == 8_000_000
    assert r["traffic_gbs"] == pytest.approx(4000.0)
    assert r["traffic_frac"] == pytest.approx(0.5)
    r = bench.add_traffic({"kernel": "k_bin", "avg_launch_us": 2.0}, "campaign")
    assert r["traffic"] is None and "traffic_gbs" not in r


def test_committed_traffic_layout(bench):
    """profiles/traffic.json: a hash of the kernel sources it was taken on, the
    copy calibration, and one table per benchmarked workload."""
    t = json.load(open(bench.TRAFFIC_FILE))
    assert len(t["kernels_hash"]) == 16
    assert t["fetch_scale"] > 0 and t["write_scale"] > 0
    for w in ("campaign", "single_pulse_10um"):
        assert t["workloads"][w]["per_launch_bytes"]["k_pairs_sp"] > 0
