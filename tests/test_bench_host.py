"""Host-side logic of bench.py (no GPU): the roofline object's arithmetic, the rule that
measured counters are used only when they were taken on the current kernel sources, and the
refusal of more than one GPU before anything touches a device."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_fields():
    r = bench.roofline(8e9, 1.0, 4e9, valu_issue=0.5, kernel="k")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(8000.0) and r["frac"] == pytest.approx(1.0)
    assert r["traffic"] == 4e9
    assert r["measured_gbs"] == pytest.approx(4000.0) and r["measured_frac"] == pytest.approx(0.5)
    assert r["valu_issue_frac"] == 0.5 and r["kernel"] == "k"
    stale = bench.roofline(8e9, 2.0, None)
    assert stale["frac"] == pytest.approx(0.5)
    assert stale["traffic"] is None and stale["measured_gbs"] is None and stale["measured_frac"] is None


@pytest.mark.parametrize("config", ["cone512", "fan512", "d4_fan512"])
def test_measured_counters_only_for_their_kernel_hash(config):
    with open(os.path.join(ROOT, "profiles", f"traffic_{config}.json")) as f:
        rec = json.load(f)
    h = rec["kernel_hash"]
    for phase, v in rec["bytes_per_launch"].items():
        assert bench.measured_traffic(h, config, phase) == v
        assert bench.measured_traffic("0" * 16, config, phase) is None
    for phase, v in rec.get("valu_issue", {}).items():
        assert bench.measured_traffic(h, config, phase, key="valu_issue") == v
        assert 0.0 < v <= 1.0
    assert bench.measured_traffic(h, "no_such_workload", "update") is None


def test_kernel_hash_covers_sources_and_tiling():
    h = bench.kernel_source_hash(bench.KERNEL_SOURCES_3D)
    assert h != bench.kernel_source_hash(bench.KERNEL_SOURCES_3D, 1 << 23)
    assert h != bench.kernel_source_hash(bench.KERNEL_SOURCES_2D)
    assert len(h) == 16
    # the host code that sets launch shapes is part of every hashed set
    assert "wamct_api3.hip" in bench.KERNEL_SOURCES_3D and "wamct_api.hip" in bench.KERNEL_SOURCES_2D


def test_more_than_one_gpu_is_refused_before_any_device_work():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr
    assert res.stdout == ""
