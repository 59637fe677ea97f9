"""Host-side contract of bench.py (no GPU): it refuses more than one GPU, and it
reports HBM traffic from the committed counter summary only while the kernel
sources that summary was measured on are unchanged."""
import json
import os
import subprocess
import sys

import bench
from paper_2211_09958_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _write_summary(root, families):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "traffic.json"), "w") as f:
        json.dump({"families": families}, f)


def test_traffic_scales_the_measured_ratio(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("fft_x", 1000.0) is None            # no summary
    _write_summary(str(tmp_path), {
        "fft_x": {"sources_sha256": rs.sources_sha256("fft_x"), "measured_over_algorithmic": 1.25},
        "grad_z": {"sources_sha256": "0" * 64, "measured_over_algorithmic": 2.0},
    })
    assert bench.traffic_for("fft_x", 1000.0) == 1250.0
    assert bench.traffic_for("grad_z", 1000.0) is None          # measured on other sources
    assert bench.traffic_for("gather", 1000.0) is None          # family not measured


def test_committed_summary_names_known_families():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        data = json.load(f)
    assert set(data["families"]) <= set(bench.FAMILY_KERNELS)
    for entry in data["families"].values():
        assert entry["measured_over_algorithmic"] > 0.5
        assert len(entry["sources_sha256"]) == 64
