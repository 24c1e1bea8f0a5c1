"""The benchmark's command-line contract: one JSON line with the fields the
harness reads, one GPU only, and refusals before any device work."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def run(*args, timeout=600):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True, timeout=timeout, cwd=ROOT)


@pytest.mark.parametrize("args", [("--gpus", "2"), ("--gpus", "8"), ("--mutual", "--precision", "mixed"),
                                  ("--mutual", "m2l", "--workload", "batch256_p6", "--precision", "fp64")])
def test_refusals_exit_before_device_work(args):
    r = run(*args, timeout=120)
    assert r.returncode == 2, r.stderr
    assert r.stdout == "" and "bench.py:" in r.stderr


@pytest.mark.gpu
def test_one_json_line_with_every_field():
    r = run("--workload", "uniform4k_p4", "--steps", "2", "--warmup", "1", "--no-cpu")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["higher_is_better"] is True
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["data"] == "synthetic"
    assert d["config"]["workload"] == "uniform4k_p4" and d["config"]["n"] == 4096
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in d["roofline"], k
    assert d["error"]["phi_rel_l2"] < 1e-2   # p = 4 against the direct sum
