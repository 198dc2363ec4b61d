"""bench.py end to end on the GPU, at a small size: one JSON line on stdout with
the fields of the benchmark record, a throughput consistent with its own time per
step, and a roofline of the dominant stage kernel."""
import json
import math
import os
import subprocess
import sys

import pytest

from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_record_small_well():
    need_gpu()
    announce("bench", "well 64^3, 4 steps")
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "64", "--steps", "4", "--warmup", "1",
           "--tile-depth", "16", "--no-cpu", "--no-fp64", "--no-batch", "--no-serve", "--no-large"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["metric"] == "cell-updates/s" and d["unit"] == "cell-updates/s"
    assert d["n_gpus"] == 1 and d["steps"] == 4 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["dtype"] == "f32" and d["data"] == "synthetic"
    assert "64^3" in d["config"]["workload"]
    # value = cells x steps / timed region, and ms_per_step = timed region / steps
    cells = 64 ** 3
    assert math.isclose(d["value"], cells / (d["ms_per_step"] * 1e-3), rel_tol=1e-3)
    rl = d["roofline"]
    assert rl["bound"] in ("hbm", "alu")
    assert rl["unit"] == ("GB/s" if rl["bound"] == "hbm" else "TFLOP/s")
    assert rl["peak"] == (8000.0 if rl["bound"] == "hbm" else pytest.approx(157.3))
    assert 0.0 < rl["frac"] < 1.0
    assert math.isclose(rl["frac"], rl["achieved"] / rl["peak"], rel_tol=1e-2)
    assert set(rl["kernels"]) == {"stage_p", "stage_c", "stage_e"}
    # the dominant kernel is the one with the longest average launch
    longest = max(rl["kernels"], key=lambda k: rl["kernels"][k]["avg_ms"])
    assert rl["kernel"] == "k_" + longest
    # no counter summary exists for this size: traffic is not claimed
    assert rl["traffic"] is None
