"""bench.py on the GPU with few steps and small CPU samples: the one JSON line
it prints carries every key of its contract, a throughput consistent with its
step time, the roofline object of the dominant kernel and the CPU baseline."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_contract():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1",
           "--cpu-sample-steps", "256", "--cpu-sample-ct", "1", "--cpu-sample-tf", "4096",
           "--cpu-reps", "1", "--cpu-batched-segs", "64"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=110, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    line = r.stdout.strip().splitlines()[-1]
    b = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in b, k
    assert b["n_gpus"] == 1 and b["steps"] == 3 and b["warmup"] == 1
    assert b["higher_is_better"] is True and b["data"] == "synthetic"
    T = b["config"]["T"]
    assert abs(b["value"] - T / (b["ms_per_step"] * 1e-3)) <= 1e-6 * b["value"]
    rf = b["roofline"]
    assert rf["bound"] in ("hbm", "alu", "mfma")
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-2)
    assert rf["unit"] == ("GB/s" if rf["bound"] == "hbm" else "TFLOP/s")
    cb = b["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    assert cb["speedup_fwd_adjoint"] > 0 and cb["speedup_plain_scan"] > 0
    assert b["batched"]["cpu_baseline"]["all_cores"]["cores"] >= 1
    for k in ("two_filter", "exact_dynamics", "coordinated_turn", "batched"):
        o = b[k]
        assert o["ms_per_step"] > 0 and o["value"] > 0 and "roofline" in o, k
        assert o["cpu_baseline"]["kind"] == "oracle", k
