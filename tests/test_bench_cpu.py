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


def test_b_iter_by_counting():
    """The algorithmic bytes of one iteration, tallied array by array on the smallest builder instance:
    B_iter = 4 nnz + 4 (P + 1) + 16 P + 16 D + 40 E, split into the demand step and the link step."""
    inst = W.parking_lot(3)
    P, D, E, nnz = inst.n_paths, inst.n_demands, inst.n_links, inst.nnz
    # demand step: int32 link ids, int32 row pointers, FP32 x and u_neg each read and written,
    # per demand FP32 D, u_dem read and written, int32 range pointer
    dem = 4 * nnz + 4 * (P + 1) + 2 * 4 * 2 * P + (4 + 2 * 4 + 4) * D
    # link step: FP32 C, g and q each read and written, int32 n_e, the FP64 load written and read
    link = (4 + 2 * 4 + 2 * 4 + 4 + 2 * 8) * E
    assert bench.b_iter_shares(inst) == (dem, link)
    assert sum(bench.b_iter_shares(inst)) == 4 * nnz + 4 * (P + 1) + 16 * P + 16 * D + 40 * E


def test_layout_bytes_by_counting():
    """This build's own bytes per launch, both link-sum variants, on the smallest builder instance."""
    inst = W.parking_lot(3)
    P, D, E, nnz = inst.n_paths, inst.n_demands, inst.n_links, inst.nnz
    for hop in (0, 4):
        ids = 2 * nnz if hop else 4 * (P + 1) + 4 * nnz
        base = ids + (8 + 8) * 2 * P + 16 * E + (4 + 8 + 2 * 8 + 2 * 8) * D
        priv = dict(hop_slots=hop, link_sums=3, scatter_workgroups=3, list_entries=0)
        rows = 3 * 8 * E
        assert bench.layout_bytes(inst, priv) == (base + rows, rows + 2 * 16 * E + 8 * E + 8 * E)
        lists = dict(hop_slots=hop, link_sums=1, scatter_workgroups=3, list_entries=640)
        assert bench.layout_bytes(inst, lists) == (base + rows + 2 * 640, rows + 2 * 16 * E + 8 * E + 8 * E)
        csc = dict(hop_slots=hop, link_sums=2, scatter_workgroups=0)
        assert bench.layout_bytes(inst, csc) == (base, 4 * nnz + 8 * P + 2 * 16 * E + 8 * E + 8 * E)


def test_profiled_kernel_names():
    """The names rocprofv3 gives the per-iteration kernels (template arguments included), which key the
    traffic summaries under profiles/."""
    assert bench.profiled_name("k_demand", 1) == "k_demand"
    assert bench.profiled_name("k_demand", 2) == "k_demand_multi<2>"
    assert bench.profiled_name("k_demand_scatter", 2, True) == "k_demand_scatter<2, true>"
    assert bench.profiled_name("k_demand_scatter", 1, False) == "k_demand_scatter<1, false>"
    assert bench.profiled_name("k_link_reduce", 2, True) == "k_link_reduce"


def test_roofline_fractions():
    inst = W.parking_lot(3)
    info = dict(hop_slots=4, link_sums=1, scatter_workgroups=2)
    names, k, it = bench.roofline_of(inst, info, 1e-3, 1e-3)
    assert names == ("k_demand_scatter", "k_link_reduce")
    a_dem, a_link = bench.b_iter_shares(inst)
    assert k["k_demand_scatter"]["achieved_gbs"] == round(a_dem / 1e-6 / 1e9, 2)
    assert it["frac"] == round((a_dem + a_link) / 2e-6 / 1e9 / bench.HBM_PEAK_GBS, 5)


def test_optimality_metric_special_cases():
    assert bench.optimality([1.0, 2.0], [1.0, 2.0], 1e-9) == 1.0
    assert bench.optimality([0.5, 4.0], [1.0, 2.0], 1e-9) == pytest.approx(0.75)
    # an optimum of zero counts as theta: any rate at or above theta scores 1
    assert bench.optimality([1e-3, 0.0], [0.0, 1.0], 1e-6) == pytest.approx(0.5)
