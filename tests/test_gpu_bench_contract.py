"""bench.py on the GPU, run as a child process with one timed step: the
one JSON line it prints carries every field of the benchmark contract
(metric, value, unit, steps, timing, dtype, config, roofline with its peak
and fraction, and the oracle's CPU baseline with its core count), and the
default workload's line its comparison legs and horizon accuracy."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [x for x in r.stdout.splitlines() if x.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    return json.loads(lines[0])


def check_line(d, steps):
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["metric"] == "cell-stage updates/s" and d["unit"] == "cell-stage/s"
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["higher_is_better"] is True
    assert d["value"] > 1e9 and d["ms_per_step"] > 0
    assert d["data"] == "synthetic" and d["vs_baseline"] is None
    assert "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert 0 < r["achieved"] < r["peak"] and r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["traffic"] is None or r["traffic"] > 0


def test_single_grid_line():
    d = run_bench("--workload", "spitzer_256", "--steps", "1", "--warmup", "0")
    check_line(d, 1)
    assert d["dtype"] == "f64" and d["config"]["grid"] == [256, 256, 256]
    # value = cells x the stages of the timed super-steps / their wall time
    per = d["config"]["stages_per_step"]
    assert len(per) == 1 and per[0] == d["config"]["stages"] and 15 <= per[0] <= 16
    assert d["value"] == pytest.approx(256 ** 3 * sum(per) / (d["ms_per_step"] * d["steps"] / 1e3), rel=1e-9)
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["unit"] == "cell-stage/s"
    assert cb["serial"]["cores"] == 1 and cb["serial"]["value"] > 0
    acc = d["accuracy"]
    assert acc["stages"]["library"] == acc["stages"]["oracle"]
    assert len(acc["rel_l1_per_step"]) == 10 and acc["first_step"]["rel_l1"] <= 1e-12
    k = acc["fp64_library"]["steps_within_1e-12"]
    assert k >= 3 and max(acc["rel_l1_per_step"][:k]) <= 1e-12


def test_default_line_is_the_768_mixed_workload():
    d = run_bench("--steps", "1", "--warmup", "0")
    check_line(d, 1)
    assert d["config"]["workload"] == "tangled3d_768_mixed_sat" and d["config"]["grid"] == [768] * 3
    assert d["config"]["precision"] == "mixed" and d["config"]["saturation"] == "central"
    legs = d["legs"]
    assert legs["fp64_plain_768"]["value"] > 0 and legs["fp64_plain_768"]["dt_hyp_same"]
    assert legs["mixed_over_fp64_768"] == pytest.approx(d["value"] / legs["fp64_plain_768"]["value"])
    for k in ("patches_2000_mixed_batched", "patches_2000_fp64_loop"):
        assert legs[k]["value"] > 0
    acc = d["accuracy"]
    assert acc["stages"]["library"] == acc["stages"]["oracle"] and len(acc["rel_l1_per_step"]) == 20
    assert acc["first_step"]["rel_l1"] <= 1e-5
    k = acc["fp64_library"]["steps_within_1e-12"]
    assert k >= 3 and max(acc["rel_l1_per_step"][:k]) <= 1e-5
    assert d["cpu_baseline"]["cores"] >= 1 and d["cpu_baseline"]["serial"]["cores"] == 1


def test_batched_line():
    d = run_bench("--workload", "patches_2000", "--steps", "1", "--warmup", "0", "--no-cpu-baseline")
    check_line(d, 1)
    assert d["config"]["patches"] == 2000 and 0 <= d["config"]["tile_policy"]
