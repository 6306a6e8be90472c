"""The benchmark's command-line contract: one JSON line with the required keys."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
        "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"}


def _run(*args, timeout=600):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=timeout)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2", timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


@pytest.mark.gpu
def test_json_line_has_the_required_keys():
    r = _run("--steps", "2", "--warmup", "1", "--targets", "200000", "--no-cpu-baseline", "--no-gate")
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert KEYS <= set(line)
    assert line["n_gpus"] == 1 and line["steps"] == 2 and line["warmup"] == 1 and line["value"] > 0
    rl = line["roofline"]
    assert {"bound", "achieved", "peak", "unit", "frac", "traffic"} <= set(rl)
    assert rl["bound"] == "hbm" and rl["peak"] == 8000.0 and 0 < rl["frac"] < 1
    assert line["config"]["workload"].startswith("gd3d") and line["accuracy_vs_truth"]["n"] == 2000
