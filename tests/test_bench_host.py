"""Host-side logic of bench.py (no GPU): the one-GPU guard, the byte model, the
sweeps-per-launch parse, the counter-summary lookup and the oracle baseline's
report fields."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import meshgen  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_sweep_bytes_counts_each_stream_once():
    # x and y of every vertex read (2*s*n), of every free vertex written
    # (2*s*n_free), 4*(n+1) row offsets, 4*nnz column ids
    assert bench.sweep_bytes(10, 7, 30, 8) == 2 * 8 * 10 + 2 * 8 * 7 + 4 * 11 + 4 * 30
    assert bench.sweep_bytes(10, 7, 30, 4) == 2 * 4 * 10 + 2 * 4 * 7 + 4 * 11 + 4 * 30


def test_sweeps_per_launch_reads_the_blocking_depth():
    assert bench.sweeps_per_launch("tb/ts256/k2/bs256/w8/r2/l1024/xcd16") == 2
    assert bench.sweeps_per_launch("tb/ts512/k4/bs512/w8/r8/l4096/linear") == 4
    assert bench.sweeps_per_launch("halo/ts256/w8/xcd") == 1
    assert bench.sweeps_per_launch("ell2/bs128/w8/r2/linear") == 1


def test_sweep_variant_reads_the_scheme_s_name():
    cfg = ("tb/ts1024/k4/bs1024/w8/r2/l2048/xcd16/patch halo/ts256/w8/xcd stop=tb/ts512/k2/bs512/w8/r2/l1024/linear"
           " colour=mc/ts1024/k2/bs512/r4/l4096/linear/patch colour_stop=mc/ts512/k1/bs256/r4/l2048/xcd16/patch"
           " tuned[0:1.00us 1:2.00us]")
    assert bench.sweep_variant(cfg) == "tb/ts1024/k4/bs1024/w8/r2/l2048/xcd16/patch"
    assert bench.sweep_variant(cfg, "multicolor") == "mc/ts1024/k2/bs512/r4/l4096/linear/patch"
    assert bench.sweep_variant("halo/ts256/w8/xcd colour=by-colour tuned[]", "multicolor") == "by-colour"
    assert bench.sweep_variant("", "multicolor") == "colour"


def test_roofline_scales_bytes_and_time_by_the_depth():
    r = dict(sweep_kernel="tb/ts256/k2/bs256/w8/r2/l1024/xcd16", bytes_per_sweep=12_000_000, sweep_us_events=3.0)
    roof = bench.roofline_of(r, "f64", "no-such-workload")
    assert roof["bytes_per_launch"] == 24_000_000 and roof["avg_launch_us"] == 6.0
    assert roof["achieved"] == pytest.approx(4000.0)                 # 24 MB in 6 us
    assert roof["frac"] == pytest.approx(0.5) and roof["traffic"] is None and roof["bound"] == "hbm"
    assert roof["launch_duration"] == "whole call" and "traffic_gbs" not in roof
    # a measured marginal launch duration takes precedence over the call's time per launch
    roof = bench.roofline_of(dict(r, launch_us_marginal=5.0), "f64", "no-such-workload")
    assert roof["avg_launch_us"] == 5.0 and roof["avg_launch_us_whole_call"] == 6.0
    assert roof["achieved"] == pytest.approx(4800.0) and roof["launch_duration"] == "marginal"


def test_roofline_reports_the_physical_rate_when_counters_exist(tmp_path, monkeypatch):
    name = "tb/ts256/k2/bs256/w8/r2/l1024/xcd16"
    summary = tmp_path / "c.md"
    summary.write_text(f"- source_sha256: {bench.device_source_hash()}\n\n| `{name}` | f64 | 1.0 / 2.0 | 600 | 0.3 |  |\n")
    monkeypatch.setitem(bench.COUNTERS, "toy", str(summary))
    r = dict(sweep_kernel=name, bytes_per_sweep=1000, sweep_us_events=3.0)
    roof = bench.roofline_of(r, "f64", "toy")
    assert roof["traffic"] == 600.0
    assert roof["traffic_gbs"] == pytest.approx(600 / 6e-6 / 1e9)      # 600 bytes in 2 x 3 us
    assert roof["traffic_per_algorithmic_byte"] == pytest.approx(0.3)


def test_counter_summary_is_used_only_for_the_current_source(tmp_path):
    row = "| `tb/ts256/k2/bs256/w8/r2/l1024/xcd16` | f64 | 1.0 / 2.0 | 84461085 | 1.014 |  |\n"
    good = tmp_path / "good.md"
    good.write_text(f"- source_sha256: {bench.device_source_hash()}\n\n" + row)
    stale = tmp_path / "stale.md"
    stale.write_text("- source_sha256: " + "0" * 64 + "\n\n" + row)
    name = "tb/ts256/k2/bs256/w8/r2/l1024/xcd16"
    assert bench.counters_traffic(name, "f64", str(good)) == 84461085.0
    assert bench.counters_traffic(name, "f32", str(good)) is None
    assert bench.counters_traffic("halo/ts256/w8/xcd", "f64", str(good)) is None
    assert bench.counters_traffic(name, "f64", str(stale)) is None
    assert bench.counters_traffic(name, "f64", str(tmp_path / "missing.md")) is None


def test_oracle_baseline_reports_its_sample():
    m = meshgen.jittered_grid(40, seed=1)
    cpu, top = bench.cpu_baseline(m, 3, budget_s=0.0, one_core_s=0.0)
    free = int((top.fixed == 0).sum())
    assert cpu["kind"] == "oracle" and cpu["unit"] == "vertex-updates/s"
    assert 1 <= cpu["cores"] <= 16 and cpu["value"] > 0 and cpu["one_core_value"] > 0
    assert cpu["cores"] <= cpu["affinity_cpus"] <= cpu["host_logical_cpus"]
    assert f"{m.n} vertices" in cpu["sample"] and free > 0
    # every ordering is timed, on all threads and on one, with the paper's gain metric
    assert set(cpu["per_ordering"]) == {"rdr", "ori", "bfs", "random"}
    for row in cpu["per_ordering"].values():
        assert row["all"]["value"] > 0 and row["one_core"]["threads"] == 1
    assert set(cpu["rdr_gain_all"]) == {"ori", "bfs", "random"}
    assert cpu["value"] == cpu["per_ordering"]["rdr"]["all"]["value"]
    assert np.isfinite(cpu["value"])


def test_relabelled_mesh_sweeps_to_the_same_positions():
    # the oracle's view of an ordering: after the inverse permutation, a sweep
    # gives the input-label result (sums reordered, so within rounding)
    from oracle import mesh as omesh
    from oracle import orderings as oord
    from oracle import smooth as osm
    m = meshgen.jittered_grid(30, seed=2, land_fraction=0.3)
    top0 = omesh.topology(m.n, m.tri)
    ex, ey = osm.jacobi(top0, m.x, m.y, 4)
    p = oord.random_order(m.n, 5)
    top, x, y = bench.relabelled(m, top0, p)
    gx, gy = osm.jacobi(top, x, y, 4)
    inv = oord.inverse(p)
    assert np.max(np.abs(gx[inv] - ex)) <= 1e-14 and np.max(np.abs(gy[inv] - ey)) <= 1e-14


def test_pass_floor_fraction_charges_one_sweep_per_launch():
    r = dict(sweep_kernel="tb/ts1024/k4/bs1024/w8/r2/l2048/xcd16/patch", bytes_per_sweep=8_000_000,
             sweep_us_events=1.0, launch_us_marginal=4.0)
    roof = bench.roofline_of(r, "f64", "no-such-workload")
    assert roof["frac"] == pytest.approx(4 * 8e6 / 4e-6 / 1e9 / 8000)
    assert roof["frac_pass_floor"] == pytest.approx(8e6 / 4e-6 / 1e9 / 8000)
    assert roof["pass_floor_bytes"] == 8_000_000
