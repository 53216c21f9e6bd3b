"""bench.py's output contract: one JSON line with the metric, the roofline of the
dominant kernel and the CPU oracle baseline; more than one GPU is refused."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


@pytest.mark.gpu
def test_short_bench_line_has_the_contract_fields():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20", "--warmup", "2", "--pass-reps", "3",
           "--adjoint-steps", "0", "--lab-steps", "0", "--unfused-steps", "0", "--plan", "8,8",
           "--cpu-sample-steps", "2", "--only-primary"]
    print("case bench.py", " ".join(cmd[2:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 2 and d["dtype"] == "f32"
    assert d["value"] > 0 and d["config"]["workload"] == "2d-512-ts4" and d["config"]["finite"]
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12 and 0 < rf["frac"] < 1
    # achieved = algorithmic bytes per launch / average launch duration
    assert abs(rf["achieved"] - rf["algorithmic_bytes_per_launch"] / (rf["avg_launch_ms"] * 1e-3) / 1e9) < 1e-6
    assert rf["copy_ceiling"]["GB_per_s"] > 0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
    assert "cpu_model" in cb and cb["one_core"]["cores"] == 1 and cb["one_core"]["value"] > 0


@pytest.mark.gpu
def test_default_bench_line_carries_every_leg():
    # the default run adds the complex128 state, the 3D 128^3 workload in both element
    # types and the ensemble, each with its own roofline, fwd+adjoint and error against
    # the oracle (short runs here)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "8", "--warmup", "2", "--pass-reps", "2",
           "--adjoint-steps", "4", "--K", "2", "--lab-steps", "0", "--unfused-steps", "0", "--plan", "default",
           "--cpu-sample-steps", "1"]
    print("case bench.py", " ".join(cmd[2:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert d["error_vs_oracle"]["rel_l2"] < 1e-5 and d["error_vs_oracle"]["steps"] == 1
    assert d["fwd_adjoint"]["grad_finite"]
    for key, wl, tol in (("2d_c128", "2d-512-ts4", 1e-12), ("3d_c64", "3d-128-ts4", 1e-5),
                         ("3d_c128", "3d-128-ts4", 1e-12)):
        leg = d[key]
        assert leg["workload"] == wl and leg["value"] > 0 and leg["finite"]
        rf = leg["roofline"]
        assert abs(rf["achieved"] - rf["algorithmic_bytes_per_launch"] / (rf["avg_launch_ms"] * 1e-3) / 1e9) < 1e-6
        assert 0 < rf["frac"] < 1 and leg["bytes_model"]["GB_per_s"] > 0
        assert leg["fwd_adjoint"]["grad_finite"] and leg["fwd_adjoint"]["value"] > 0
        assert leg["error_vs_oracle"]["rel_l2"] < tol, (key, leg["error_vs_oracle"])
    assert d["ensemble"]["value"] > 0 and d["ensemble"]["finite"] and d["ensemble"]["fwd_adjoint"]["value"] > 0
