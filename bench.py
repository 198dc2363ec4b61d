"""Benchmark of the CSPH-TVD step on one MI355X.

Workload (default): supersonic flow through a Gaussian potential well on a 256^3
grid (psi = -exp(-r^2/0.01), gamma = 5/3, Mach-2 inflow), FP32 state.  A step is
one full CSPH-TVD step (Lagrangian predictor + corrector, Eulerian remap, CFL
dt) of every interior cell; the metric is cell-updates/s = cells * steps / time,
with the state resident in HBM before the timed region starts.

Prints one JSON line.  Besides the headline it carries:
  roofline     -- the dominant kernel's algorithmic bytes per launch over its
                  average launch time (HIP events recorded by the library
                  around each kernel during the timed steps), against 8 TB/s;
  cpu_baseline -- the FP64 CPU oracle timed on this host (rank 0 only) on a
                  bounded sample of the same workload;
  fp64         -- the same workload with FP64 state, timed the same way.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # bytes/s, MI355X

# Algorithmic bytes per interior cell of each stage kernel, in words (4 B in
# FP32, 8 B in FP64): every input read once, every output written once.
#   stage P: read U^n (5) + psi (1);            write m*, E* (4) + xi* (3)
#   stage C: read rho, m*, E* (5) + xi* (3) + psi (1) + m^n, E^n (4); write m~, E~ (4) + xi (3)
#   stage E: read U^n (5) + m~, E~ (4) + xi (3); write U^{n+1} (5)
WORDS = {"stage_p": 13, "stage_c": 20, "stage_e": 17}
KERNEL_NAMES = {"stage_p": "k_stage_p", "stage_c": "k_stage_c", "stage_e": "k_stage_e"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(prob, dtype, steps, warmup):
    import torch
    from paper_1912_04855_amd.sim import from_problem

    sim = from_problem(prob, dtype=dtype, torch=True)
    stream = torch.cuda.current_stream()
    if warmup:
        sim.advance(math.inf, warmup)
    torch.cuda.synchronize()
    sim.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    n = sim.advance(math.inf, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    prof = sim.profile_read()
    sim.profile(False)
    assert n == steps, (n, steps)
    t, nsteps = sim.time()
    sim.close()
    return {"wall_s": wall, "event_ms": gpu_ms, "profile": prof, "t": t}


def roofline(prof, cells, dtype):
    word = 8 if dtype == "f64" else 4
    dom = max(WORDS, key=lambda k: prof[k][0])
    ms = prof[dom][0]
    bytes_per_launch = WORDS[dom] * word * cells
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    per = {k: {"avg_ms": round(prof[k][0], 5), "launches": prof[k][1],
               "GBps": round(WORDS[k] * word * cells / (prof[k][0] * 1e-3) / 1e9, 1)}
           for k in WORDS}
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            rec = json.load(open(tf)).get(f"{KERNEL_NAMES[dom]}:{dtype}:{cells}")
            if rec and rec.get("source_hash") == source_hash():
                traffic = rec["bytes_per_launch"]
        except Exception:
            traffic = None
    return {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": round(achieved, 1),
            "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(achieved * 1e9 / HBM_PEAK, 4),
            "traffic": traffic, "bytes_per_launch": bytes_per_launch, "kernels": per}


def source_hash():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1912_04855_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(budget_s=15.0):
    """The FP64 oracle (single thread) on a 64^3 sample of the same workload."""
    import oracle as O
    from paper_1912_04855_amd import problems as P

    pr = P.well_flow(64)
    s = O.OracleSim(pr.shape, pr.h, gamma=pr.gamma, cfl=pr.cfl, rho_vac=pr.rho_vac, bc=pr.bc,
                    inflow=pr.inflow_list())
    s.set_primitive(pr.prim)
    s.set_potential(pr.psi)
    t0 = time.perf_counter()
    n = 0
    while n < 3 or (time.perf_counter() - t0 < budget_s and n < 200):
        s.step()
        n += 1
    el = time.perf_counter() - t0
    return {"value": round(pr.cells * n / el, 1), "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"potential-well flow 64^3 (same setup rescaled), {n} FP64 steps, "
                      f"single-threaded C oracle, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="grid edge of the potential-well workload")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 companion run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (reference for the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the multi-GPU decomposition is not built "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {n} bytes 5 times")
        return
    from paper_1912_04855_amd import problems as P

    pr = P.well_flow(args.n, steps=args.steps)
    cells = pr.cells
    log(f"[bench] potential-well flow {args.n}^3 {args.dtype}: warmup {args.warmup}, "
        f"{args.steps} timed steps")
    r = run_gpu(pr, args.dtype, args.steps, args.warmup)
    ms_step = r["event_ms"] / args.steps
    value = cells * args.steps / (r["event_ms"] * 1e-3)
    log(f"[bench] {ms_step:.3f} ms/step, {value:.3e} cell-updates/s "
        f"(wall {r['wall_s']:.3f} s)")
    rl = roofline(r["profile"], cells, args.dtype)
    out = {
        "metric": "cell-updates/s", "value": round(value, 1), "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"potential-well flow {args.n}^3 (Mach-2 inflow, "
                               f"psi=-exp(-r^2/0.01), gamma=5/3)",
                   "cells": cells, "dtype": args.dtype, "parallelism": "single GPU"},
        "roofline": rl,
        "algorithmic_hbm_frac": round(value * (44 if args.dtype == "f32" else 88) / HBM_PEAK, 4),
    }
    if not args.no_fp64 and args.dtype == "f32":
        k64 = max(10, args.steps // 2)
        log(f"[bench] FP64 companion: {k64} steps")
        r64 = run_gpu(pr, "f64", k64, args.warmup)
        v64 = cells * k64 / (r64["event_ms"] * 1e-3)
        out["fp64"] = {"value": round(v64, 1), "ms_per_step": round(r64["event_ms"] / k64, 4),
                       "steps": k64, "roofline": roofline(r64["profile"], cells, "f64")}
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
