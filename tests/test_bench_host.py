"""Host-side logic of bench.py (no GPU): the one-GPU guard, the tile-depth
argument, the roofline arithmetic of the dominant kernel, each kernel's bound
from its measured VALU-busy share, and that counter summaries are used only for
the source they were taken of."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

CELLS = 256 ** 3


def _prof(p, c, e):
    return {"stage_p": (p, 100), "stage_c": (c, 100), "stage_e": (e, 100),
            "ghost_fill": (0.02, 300), "bookkeeping": (0.003, 200)}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_tile_depth_argument():
    assert bench._depths("16") == 16
    assert bench._depths("64,16,32") == (64, 16, 32)
    with pytest.raises(Exception):
        bench._depths("8,8")
    assert bench._tile((64, 16, 32)) == "P/C 64x4, E 32x8, z-depth P/C/E 64/16/32"
    assert bench._tile((8, 8, 8), "f64") == "32x8, z-depth P/C/E 8/8/8"


def test_roofline_of_an_hbm_bound_kernel(monkeypatch):
    monkeypatch.setattr(bench, "_counters", lambda *a: None)
    r = bench.roofline(_prof(0.3, 0.4, 0.5), CELLS, "f32", stream_gbps=5000.0)
    # the longest launch is stage E: 12 reads + 5 writes of 4 B per cell
    assert r["kernel"] == "k_stage_e" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    gbps = 17 * 4 * CELLS / 0.5e-3 / 1e9
    assert r["achieved"] == pytest.approx(gbps, abs=0.06)
    assert r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(gbps / 8000.0, abs=1e-4)
    assert r["traffic"] is None
    assert r["hbm"]["bytes_per_launch"] == 17 * 4 * CELLS
    assert r["hbm"]["stream_reference"]["frac"] == pytest.approx(gbps / 5000.0, abs=1e-4)
    # every stage kernel is listed with its own bound and rate; without a counter
    # summary of the current source the last measured bounds stand
    assert set(r["kernels"]) == {"stage_p", "stage_c", "stage_e"}
    assert r["kernels"]["stage_p"]["bound"] == "alu" and r["kernels"]["stage_c"]["bound"] == "hbm"
    assert r["kernels"]["stage_p"]["valu_busy"] is None
    assert r["kernels"]["stage_p"]["GBps"] == pytest.approx(12 * 4 * CELLS / 0.3e-3 / 1e9, abs=0.06)
    assert r["other_kernels"]["ghost_fill"]["launches"] == 300


def test_bound_follows_measured_valu_busy(monkeypatch):
    busy = {"k_stage_p": 0.81, "k_stage_c": 0.9, "k_stage_e": 0.65}
    monkeypatch.setattr(bench, "_counters", lambda k, d, c: {"valu_busy": busy[k],
                                                             "bytes_per_launch": None})
    r = bench.roofline(_prof(0.3, 0.6, 0.5), CELLS, "f32")
    # stage C has the longest launch and its VALU is busy 90% of it: ALU-bound
    assert r["kernel"] == "k_stage_c" and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["valu_busy"] == 0.9
    tf = 411 * CELLS / 0.6e-3 / 1e12
    assert r["achieved"] == pytest.approx(tf, abs=0.006)
    assert r["peak"] == pytest.approx(157.3)
    assert r["alu"]["frac_nonpacked"] == pytest.approx(tf / 78.6, abs=1e-4)
    assert r["kernels"]["stage_e"]["bound"] == "hbm"
    assert max(k["valu_busy"] for k in r["kernels"].values()) <= 1.0
    # FP64 words are 8 bytes, and stage C moves 14 + 7 of them
    r64 = bench.roofline(_prof(1.0, 2.0, 0.9), CELLS, "f64")
    assert r64["hbm"]["bytes_per_launch"] == 21 * 8 * CELLS
    assert r64["peak"] == pytest.approx(78.6)


def test_counter_summaries_follow_the_source(monkeypatch):
    real = bench.source_hash()
    assert len(real) == 16
    monkeypatch.setattr(bench, "source_hash", lambda: "0000000000000000")
    assert bench._counters("k_stage_e", "f32", CELLS) is None
    monkeypatch.setattr(bench, "source_hash", lambda: real)
    rec = bench._counters("k_stage_e", "f32", CELLS)
    if rec is not None:
        # measured traffic of a summary taken of this source: of the order of
        # the algorithmic bytes (halos add to them), and a VALU-busy share
        alg = 17 * 4 * CELLS
        assert 0.8 * alg < rec["bytes_per_launch"] < 3.0 * alg
        assert rec["read"] + rec["written"] == pytest.approx(rec["bytes_per_launch"], rel=1e-6)
        assert 0.0 < rec["valu_busy"] <= 1.0


def test_host_description():
    d = bench.host_description()
    assert d["nproc"] >= 1 and d["usable_cpus"] >= 1
    assert d.get("model")


def test_batch_shapes_match_the_instances():
    from paper_1912_04855_amd import problems as P
    for k in range(6):
        shape, kind = P.batch_shape(0, k)
        pr = P.batch_instance(0, k, steps=3)
        assert pr.shape == shape and pr.name == kind
