"""Host-side checks of the measurement script (no GPU): it refuses more than
one GPU before touching the device, the adjoint budget arithmetic, and the
traffic record is ignored unless it matches the kernel sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_snapshot_budget_arithmetic():
    from paper_1202_6081_amd import autograd as ag
    gib = 2**30
    assert ag.binomial_snapshots_for_budget(13.5 * gib, 230 * gib, 104 * gib) == 9
    assert ag.binomial_snapshots_for_budget(10 * gib, 50 * gib, 60 * gib) == 0


def test_traffic_record_tied_to_sources(tmp_path, monkeypatch):
    import pytest
    import bench
    n = 512**3
    rec = json.load(open(bench.COUNTERS_FILE))
    assert rec["nodes"] == n
    if rec["source_hash"] != bench.kernel_source_hash():
        pytest.skip("kernel sources changed since the counters were taken (bench reports traffic null)")
    assert bench.measured_traffic(n) == rec["hbm_bytes_per_dispatch"]
    # and is ignored for another source hash or lattice size
    stale = dict(rec, source_hash="0" * 16)
    path = tmp_path / "c.json"
    path.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(path))
    assert bench.measured_traffic(n) is None
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic(256**3) is None
    # algorithmic vs measured: within 1% for the step
    assert abs(rec["hbm_bytes_per_dispatch"] / (bench.BYTES_PER_NODE * n) - 1) < 0.01


def test_cpu_baseline_reports_host_and_references():
    # The oracle's timing leg on a tiny sample: the record names the worker
    # count, the host's CPU count and model, and the untimed references of the
    # accuracy checks have the sample's shapes.
    import bench
    rec, ref = bench.cpu_baseline(seconds_target=0.2, n=8, max_steps=2, adjoint_steps=2)
    assert rec["kind"] == "oracle" and rec["unit"] == "MLUPS" and rec["value"] > 0
    assert rec["cores"] == min(os.cpu_count(), 16) and rec["host_cpus"] == os.cpu_count()
    assert "cpu_model" in rec and "worker processes" in rec["sample"]
    assert ref["f27"].shape == (27, 8, 8, 8) and ref["f15"].shape == (15, 8, 8, 8)
    assert ref["u27"].shape == (3, 8, 8, 8) and ref["steps"] >= 2
    assert ref["dL_dF_dot_v"] != 0.0 and ref["loss"] > 0.0
