"""bench.py end to end on a small lattice (64^3, a few steps): one JSON line
with the fields of its contract, every section present and self-consistent."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_small_lattice_json_line():
    print("case bench 64^3", flush=True)
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--n", "64", "--steps", "6", "--warmup",
                          "2", "--adjoint-steps", "6", "--no-cpu-baseline"], capture_output=True, text=True,
                         timeout=240, cwd=ROOT)
    assert res.returncode == 0, res.stderr[-2000:]
    lines = [l for l in res.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, res.stdout
    r = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in r, key
    assert r["n_gpus"] == 1 and r["steps"] == 6 and r["warmup"] == 2
    assert r["config"]["nodes"] == 64**3
    assert r["value"] > 0 and abs(r["value"] - 64**3 / (r["ms_per_step"] * 1e3)) <= 1e-2 * r["value"]
    roof = r["roofline"]
    assert roof["bound"] == "hbm" and roof["peak"] == 8000.0 and roof["unit"] == "GB/s"
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert roof["traffic"] is None              # counters are recorded for the 512^3 workload only
    assert r["hbm_ceiling"] is None             # the rate probe covers lattices of a multiple of 256 only
    assert len(r["variants"]) == 8 and all(v["ms"] > 0 and v["inplace"]["ms"] > 0 for v in r["variants"])
    assert [v["lattice"] for v in r["adjoint_variants"]] == ["D3Q27", "D3Q15"]
    adj = r["adjoint"]
    assert adj["adjoint_steps"] == 6 and adj["recomputed_steps"] >= 0
    assert r["adjoint_forward_ratio"] == adj["ratio_backward_over_forward_steps"] > 0


def test_hbm_probe_runs():
    # The HBM rate probe that the roofline is read against, on a 256^3 lattice.
    print("case hbm_probe 256", flush=True)
    exe = os.path.join(ROOT, "paper_1202_6081_amd", "hbm_probe")
    assert os.path.exists(exe), "hbm_probe is built by __graft_entry__.build()"
    res = subprocess.run([exe, "256"], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr[-2000:]
    r = json.loads(res.stdout.strip().splitlines()[-1])
    assert r["nodes"] == 256**3
    for key in ("read_GBs", "write_GBs", "copy_GBs", "step_traffic_pull_GBs", "step_traffic_own_node_GBs"):
        assert 100.0 < r[key] < 8000.0, (key, r[key])
    bad = subprocess.run([exe, "100"], capture_output=True, text=True, timeout=60)
    assert bad.returncode == 2                # sizes the probe's launch shape cannot cover are refused
