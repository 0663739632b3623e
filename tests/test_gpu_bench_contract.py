"""bench.py's output contract on a short run: one JSON line on stdout with the metric, the
whole-job value, exactly the step counts asked for (a step of the headline workload is one
diagnostic period of MD steps), the roofline of the Coulomb kernel (achieved over peak, the
kernel's own launch time) and, when asked, the oracle baseline on the host."""
import json
import os
import subprocess
import sys

import pytest

from _helpers import gpu_available

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_bench_json_line():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "12", "--warmup", "3", "--profile-steps", "20",
           "--no-oracle-records", "--no-cpu-baseline"]
    print(" ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 12 and d["warmup"] == 3
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["unit"] == "Gpair/s" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert "workload" in d["config"] and "model" not in d["config"]
    # the whole-job rate is the pair interactions of the timed MD steps over their wall time
    n, per = d["config"]["n_particles"], d["config"]["md_steps_per_step"]
    assert per == d["config"]["diagnostic_every"] == 100
    assert abs(d["value"] - float(n) * n * per / (d["ms_per_step"] * 1e-3) / 1e9) <= 1e-3 * d["value"]
    assert abs(d["ms_per_md_step"] * per - d["ms_per_step"]) <= 1e-3 * d["ms_per_step"]
    rf = d["roofline"]
    assert rf["bound"] in ("hbm", "mfma", "alu") and rf["unit"] in ("GB/s", "TFLOP/s")
    assert rf["peak"] == 157.3 and 0.0 < rf["frac"] < 1.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-3
    assert rf["traffic"] is None or rf["traffic"] > 0
    assert "cpu_baseline" not in d
    print(f"value {d['value']} Gpair/s, frac {rf['frac']}", flush=True)
