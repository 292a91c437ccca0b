"""Host-side checks of bench.py: the single-GPU guard, the traffic lookup keyed to the kernel sources,
and the algorithmic byte counts of the per-iteration kernels on a hand-sized instance."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _recorded_hash():
    with open(bench.TRAFFIC_FILE) as fh:
        m = re.search(r"```json\n(.*?)\n```", fh.read(), re.S)
    return json.loads(m.group(1))["kernel_sha256_16"]


def test_traffic_reported_only_for_the_profiled_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_hash", _recorded_hash)
    for k in ("k_demand", "k_link"):
        t = bench.measured_traffic(k)
        assert isinstance(t, int) and t > 0
    assert bench.measured_traffic("no_such_kernel") is None
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0" * 16)
    assert bench.measured_traffic("k_demand") is None


def test_traffic_missing_file(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.measured_traffic("k_demand") is None


def test_kernel_bytes_by_counting():
    """Byte counts of the smallest builder instance, tallied array by array from its sizes."""
    inst = W.parking_lot(3)
    P, D, E, nnz = inst.n_paths, inst.n_demands, inst.n_links, inst.nnz
    # demand kernel: link ids, x and u_neg (FP64) read and written, FP32 x written, (g, q) per link,
    # per demand: range pointer, demand, u_dem and S read and written
    for H in (0, 4, 8):
        ids = 2 * H * P if H else 4 * (P + 1) + 4 * nnz
        dem = ids + (8 + 8) * 2 * P + 4 * P + 16 * E + (4 + 8 + 2 * 8 + 2 * 8) * D
        # link kernel: CSC path ids, FP32 x, (g, q) read and written, capacity, non-empty link tables
        link = 4 * nnz + 4 * P + 2 * 16 * E + 8 * E + 8 * E
        assert bench.kernel_bytes(inst, H) == (dem, link)


def test_optimality_metric_special_cases():
    assert bench.optimality([1.0, 2.0], [1.0, 2.0], 1e-9) == 1.0
    assert bench.optimality([0.5, 4.0], [1.0, 2.0], 1e-9) == pytest.approx(0.75)
    # an optimum of zero counts as theta: any rate at or above theta scores 1
    assert bench.optimality([1e-3, 0.0], [0.0, 1.0], 1e-6) == pytest.approx(0.5)
