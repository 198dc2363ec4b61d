"""Benchmark of the CSPH-TVD step on one MI355X.

Workload (default): supersonic flow through a Gaussian potential well on a 256^3
grid (psi = -exp(-r^2/0.01), gamma = 5/3, Mach-2 inflow), FP32 state.  A step is
one full CSPH-TVD step (Lagrangian predictor + corrector, Eulerian remap, CFL
dt) of every interior cell; the metric is cell-updates/s = cells * steps / time,
with the state resident in HBM before the timed region starts.

Prints one JSON line.  Besides the headline it carries:
  roofline     -- the stage kernel with the longest launches against the bound
                  it has (HBM for stages P and E, the vector ALU for stage C):
                  algorithmic bytes (or flops) per launch over its average launch
                  time (HIP events the library records around each kernel in a
                  second pass of the timed steps), with the other view beside it,
                  the HBM traffic counted by rocprofv3, a streaming reference
                  kernel with the same mix of read and write streams, and the
                  whole step against the vector-ALU issue rate;
  cpu_baseline -- the FP64 CPU oracle timed on this host (rank 0 only) on a
                  bounded sample of the same workload;
  fp64, batched, serving -- the same workload with FP64 state; 512 uneven
                  simulations advanced together; a Poisson stream of requests.
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
# Vector ALU peaks of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x
# 2.4 GHz = 78.6 TFLOP/s for non-packed FP32 and for FP64; packed FP32 doubles
# the FP32 figure to the published 157.3 TFLOP/s.  The kernels are built with
# packed FP32 switched off, so 78.6 is the rate they can reach; the published
# figure is reported as the peak.
ALU_PEAK = {"f32": 157.3e12, "f64": 78.6e12}
ALU_PEAK_NONPACKED = 78.6e12
VALU_ISSUE = 256 * 4 * 16 * 2.4e9   # lane-instructions/s (one wave64 op per SIMD per 4 clocks)

# Algorithmic bytes per interior cell of each stage kernel, in words (4 B in
# FP32, 8 B in FP64): every input of the kernel read once, every output written
# once.  The FP32 build does not store the particle offsets xi*, xi^{n+1}: it
# forms them from the momenta where they are needed.
#   stage P: read U^n (5) + psi (1);  write m*, E* (4) + psi(r*) (1)
#            [FP64 also writes xi* (3)]
#   stage C: read rho, m*, E* (5) + psi(r*) (1) + m^n, E^n (4);  write m~, E~ (4)
#            [FP64 reads xi* (3) and writes xi^{n+1} (3)]
#   stage E: read U^n (5) + m~, E~ (4) + m* (3) [FP64: xi^{n+1} (3)];  write U^{n+1} (5)
RW = {"f32": {"stage_p": (6, 5), "stage_c": (10, 4), "stage_e": (12, 5)},
      "f64": {"stage_p": (6, 8), "stage_c": (13, 7), "stage_e": (12, 5)}}
WORDS = {t: {k: r + w for k, (r, w) in m.items()} for t, m in RW.items()}
# What bounds each kernel (rocprofv3 counters): the corrector issues vector-ALU
# instructions back to back; the predictor and the Eulerian update wait on HBM.
BOUND = {"stage_p": "hbm", "stage_c": "alu", "stage_e": "hbm"}
# Algorithmic floating-point operations per interior cell of each stage (each
# +, -, *, /, sqrt, min, max counted once; a fused multiply-add is two), as the
# method defines them, not as the kernels happen to issue them:
#   stage P: primitives (14) + the 13 lattice pair terms of A (119), D[psi] (54)
#            and B (212) + rho u.D[psi] (7) + the predictor update (20) + psi at
#            r* (27)                                                      = 453
#   stage C: per neighbour (26): separation (5), |d| and q (7), g(q)/q (4), K (4),
#            pressure-potential term (4), A (6), D[psi] (6), (u_i+u_j).K/2 (9),
#            B (2) = 47.1; plus primitives, corrector update and xi (51)  = 1275
#   stage E: three faces per cell (a face is shared by two cells) x 148 (slopes
#            and minmod 45, reconstruction and swept flux 41, acoustic damping
#            62) + the update (35) + the next step's signal speed (21) and the
#            totals (5)                                                    = 505
FLOPS = {"stage_p": 453, "stage_c": 1275, "stage_e": 505}
KERNEL_NAMES = {"stage_p": "k_stage_p", "stage_c": "k_stage_c", "stage_e": "k_stage_e"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _depths(text):
    """--tile-depth: one depth for every stage, or 'p,c,e'."""
    v = [int(x) for x in str(text).split(",")]
    if len(v) not in (1, 3):
        raise argparse.ArgumentTypeError("one depth or three (stage P, C, E)")
    return v[0] if len(v) == 1 else tuple(v)


def _tile(depths):
    """Tile shape and the z-depth of each stage's sweep."""
    return "32x8, z-depth P/C/E " + "/".join(str(d) for d in depths)


def run_gpu(prob, dtype, steps, warmup, autotune=True, tile_depth=0):
    """Warm-up, then two timed passes of `steps` steps each.  The first has HIP
    events only at its two ends and gives the throughput; the second records
    events around every kernel (an event between two kernels costs a few
    microseconds of idle time, so the first pass leaves them out) and gives each
    kernel's average launch duration."""
    import torch
    from paper_1912_04855_amd.sim import from_problem

    sim = from_problem(prob, dtype=dtype, torch=True)
    stream = torch.cuda.current_stream()
    if tile_depth:
        sim.tile_depth = tile_depth
    elif autotune:
        sim.autotune(trial_steps=3)
    tz = sim.tile_depth
    if warmup:
        sim.advance(math.inf, warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    n = sim.advance(math.inf, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    assert n == steps, (n, steps)
    # kernel durations: the same number of steps with events around each kernel
    sim.profile(True)
    n = sim.advance(math.inf, steps)
    prof = sim.profile_read()
    sim.profile(False)
    torch.cuda.synchronize()
    assert n == steps, (n, steps)
    t, nsteps = sim.time()
    sim.close()
    return {"wall_s": wall, "event_ms": gpu_ms, "profile": prof, "t": t, "tile_depth": tz}


def _counters(kernel, dtype, cells):
    """rocprofv3 counter summary of this kernel build and workload, if one was
    taken of the current kernel source (else None)."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        return None
    try:
        rec = json.load(open(tf)).get(f"{kernel}:{dtype}:{cells}")
    except Exception:
        return None
    if rec and rec.get("source_hash") == source_hash():
        return rec
    return None


def step_issue_bound(dtype, cells, ms_per_step):
    """The whole step against the vector-ALU issue rate: the counted VALU
    instructions per cell of the three stage kernels (rocprofv3 SQ_INSTS_VALU,
    committed summary of the current kernel source), each a wave64 instruction
    taking 4 clocks of one of 1024 SIMDs at 2.4 GHz.  None without a summary."""
    per = {}
    for k in WORDS[dtype]:
        rec = _counters(KERNEL_NAMES[k], dtype, cells)
        if not rec or not rec.get("valu_per_cell"):
            return None
        per[k] = rec["valu_per_cell"]
    total = sum(per.values())
    issue_ms = total * cells / VALU_ISSUE * 1e3
    return {"valu_instr_per_cell": {k: round(v, 1) for k, v in per.items()},
            "valu_instr_per_cell_total": round(total, 1), "issue_bound_ms": round(issue_ms, 4),
            "frac_of_step": round(issue_ms / ms_per_step, 3)}


def dominant(prof, dtype):
    """The stage kernel with the longest average launch."""
    return max(WORDS[dtype], key=lambda k: prof[k][0])


def stream_ceiling(kernel, dtype, cells, reps=10):
    """GB/s of a plain streaming kernel with `kernel`'s mix of read and write
    streams over the interior cells (no halos, address order): the rate HBM
    gives that mix of bytes."""
    import ctypes as C
    import torch
    from paper_1912_04855_amd import _lib
    r, w = RW[dtype][kernel]
    words = cells * (2 if dtype == "f64" else 1)
    ms = C.c_double()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = _lib.load().csph_stream_probe(r, w, words, reps, stream, C.byref(ms))
    if st != 0:
        raise RuntimeError(f"csph_stream_probe failed with status {st}")
    return (r + w) * words * 4 / (ms.value * 1e-3) / 1e9


def roofline(prof, cells, dtype, stream_gbps=None):
    """Roofline of the longest-running stage kernel against the bound it has
    (HBM bytes or vector-ALU flops), with the other view beside it; with
    `stream_gbps`, its HBM rate also against that kernel's streaming reference."""
    word = 8 if dtype == "f64" else 4
    W = WORDS[dtype]
    dom = dominant(prof, dtype)
    sec = prof[dom][0] * 1e-3
    bytes_per_launch = W[dom] * word * cells
    flops_per_launch = FLOPS[dom] * cells
    gbps = bytes_per_launch / sec / 1e9
    tflops = flops_per_launch / sec / 1e12
    rec = _counters(KERNEL_NAMES[dom], dtype, cells)
    traffic = rec["bytes_per_launch"] if rec else None
    per = {k: {"avg_ms": round(prof[k][0], 5), "launches": prof[k][1], "bound": BOUND[k],
               "GBps": round(W[k] * word * cells / (prof[k][0] * 1e-3) / 1e9, 1),
               "TFLOPs": round(FLOPS[k] * cells / (prof[k][0] * 1e-3) / 1e12, 2)}
           for k in W}
    alu = {"achieved": round(tflops, 2), "peak": ALU_PEAK[dtype] / 1e12, "unit": "TFLOP/s",
           "frac": round(tflops * 1e12 / ALU_PEAK[dtype], 4), "flops_per_launch": flops_per_launch,
           "peak_nonpacked": ALU_PEAK_NONPACKED / 1e12,
           "frac_nonpacked": round(tflops * 1e12 / ALU_PEAK_NONPACKED, 4)}
    hbm = {"achieved": round(gbps, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
           "frac": round(gbps * 1e9 / HBM_PEAK, 4), "bytes_per_launch": bytes_per_launch,
           "traffic": traffic}
    if traffic:
        hbm["traffic_GBps"] = round(traffic / sec / 1e9, 1)
    if stream_gbps:
        hbm["stream_reference"] = {
            "GBps": round(stream_gbps, 1), "frac": round(gbps / stream_gbps, 4),
            "what": "a plain kernel with the same read/write stream mix over the interior cells "
                    "(no halos, address order)"}
    main = hbm if BOUND[dom] == "hbm" else alu
    out = {"bound": BOUND[dom], "kernel": KERNEL_NAMES[dom], "achieved": main["achieved"],
           "peak": main["peak"], "unit": main["unit"], "frac": main["frac"], "traffic": traffic,
           "alu": alu, "hbm": hbm, "kernels": per,
           # the step's other launches: three ghost fills (the first timed with the
           # step's opening launch) and the closing bookkeeping launch
           "other_kernels": {k: {"avg_ms": round(prof[k][0], 5), "launches": prof[k][1]}
                             for k in ("ghost_fill", "bookkeeping") if k in prof}}
    if rec and rec.get("valu_per_cell"):
        # VALU issue utilisation from the counted instructions per cell
        out["valu_issue_frac"] = round(rec["valu_per_cell"] * cells / sec / VALU_ISSUE, 3)
    return out


def run_batch(count=512, steps=100, seed=0, chunk=10, tile_depth=0):
    """The batched workload: `count` independent simulations of uneven sizes
    (edges in {32, 48, 64, 96} per axis, a Sod tube or a Sedov blast each), FP32,
    advanced together `steps` steps each; one launch per stage for the whole
    batch, `chunk` steps per captured HIP graph."""
    import torch
    from paper_1912_04855_amd import problems as P
    from paper_1912_04855_amd.sim import Batch, from_problem

    t0 = time.perf_counter()
    sims, cells = [], 0
    b = Batch("f32")
    for k in range(count):
        pr = P.batch_instance(seed, k, steps=steps)
        s = from_problem(pr, dtype="f32")
        sims.append(s)
        cells += pr.cells
        if tile_depth:
            s.tile_depth = tile_depth
        b.add(s, steps)
    setup = time.perf_counter() - t0
    if tile_depth:
        tz = tile_depth
    else:
        tz, _ = b.autotune(trial_steps=3)
    # the batch runs on a stream of its own: the timed region is bracketed by
    # device synchronisations and measured on the host clock
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range((steps + chunk - 1) // chunk):
        b.advance(chunk, sync=False)
    done = len(b.poll())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    assert done == count, (done, count)
    for s in sims:
        t, n = s.time()
        assert n == steps, n
    b.close()
    for s in sims:
        s.close()
    return {"value": round(cells * steps / wall, 1), "unit": "cell-updates/s", "instances": count,
            "cells": cells, "steps_each": steps, "ms_per_step": round(wall * 1e3 / steps, 4),
            "tile": f"32x8, z-depth {tz}", "setup_s": round(setup, 2), "dtype": "f32",
            "workload": f"{count} instances, edges uniform in {{32,48,64,96}} per axis, "
                        "Sod tube or Sedov blast by seed"}


def run_serve(count=40, rate=1.0, seed=0, budget=64 << 30):
    """A Poisson stream of solve requests through the continuous-batching loop:
    cube edge in {64, ..., 256}, kind in {Sod, Sedov, well, cloud}, FP32 or FP64,
    50-500 steps, arriving at a fixed mean rate (requests per second).  The
    loop's capacity is measured first on a saturated burst of 8 requests and
    reported beside it (the load is rate / capacity): near full load the
    latencies of a 40-request stream are dominated by queueing and vary widely
    from run to run, so the rate is fixed rather than derived from the burst."""
    from paper_1912_04855_amd import problems as P
    from paper_1912_04855_amd import serve as S

    burst = P.serve_requests(count=8, rate=1e6, seed=seed + 1)
    st = S.serve(burst, budget_bytes=budget)
    capacity = len(burst) / st.wall_s
    reqs = P.serve_requests(count=count, rate=rate, seed=seed)
    st = S.serve(reqs, budget_bytes=budget)
    out = st.summary()
    out = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}
    out["arrival_rate_per_s"] = round(rate, 3)
    out["burst_capacity_per_s"] = round(capacity, 3)
    out["budget_bytes"] = budget
    out["workload"] = ("Poisson arrivals; cube edge in {64..256}, kind in {sod, sedov, well, "
                       "cloud}, dtype f32 or f64, 50-500 steps; latency = arrival to result on host")
    return out


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
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in tile depth instead of autotuning it first")
    ap.add_argument("--tile-depth", type=_depths, default=0,
                    help="use this tile depth (z-planes per workgroup; one value, or three "
                         "comma-separated for stages P,C,E) instead of autotuning")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched workload (for profiling it)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-tile-depth", type=int, default=0,
                    help="tile depth of every batch member instead of autotuning it")
    ap.add_argument("--serve-count", type=int, default=40)
    ap.add_argument("--serve-rate", type=float, default=1.0,
                    help="mean arrival rate of the serving workload (requests per second)")
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

    if args.batch_only:
        r = run_batch(count=args.batch_count, steps=args.steps, tile_depth=args.batch_tile_depth)
        print(json.dumps({"batched": r}), flush=True)
        return
    pr = P.well_flow(args.n, steps=args.steps)
    cells = pr.cells
    log(f"[bench] potential-well flow {args.n}^3 {args.dtype}: warmup {args.warmup}, "
        f"{args.steps} timed steps")
    r = run_gpu(pr, args.dtype, args.steps, args.warmup, autotune=not args.no_autotune,
                tile_depth=args.tile_depth)
    ms_step = r["event_ms"] / args.steps
    value = cells * args.steps / (r["event_ms"] * 1e-3)
    log(f"[bench] {ms_step:.3f} ms/step, {value:.3e} cell-updates/s "
        f"(wall {r['wall_s']:.3f} s)")
    dom = dominant(r["profile"], args.dtype)
    try:
        ref = stream_ceiling(dom, args.dtype, cells)
    except Exception as e:  # the roofline stands without the reference
        log(f"[bench] streaming reference failed: {e}")
        ref = None
    rl = roofline(r["profile"], cells, args.dtype, ref)
    sib = step_issue_bound(args.dtype, cells, ms_step)
    if sib:
        rl["step_valu_issue"] = sib
    out = {
        "metric": "cell-updates/s", "value": round(value, 1), "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"potential-well flow {args.n}^3 (Mach-2 inflow, "
                               f"psi=-exp(-r^2/0.01), gamma=5/3)",
                   "cells": cells, "dtype": args.dtype, "parallelism": "single GPU",
                   "tile": _tile(r["tile_depth"])},
        "roofline": rl,
        "algorithmic_hbm_frac": round(value * (44 if args.dtype == "f32" else 88) / HBM_PEAK, 4),
    }
    if not args.no_fp64 and args.dtype == "f32":
        k64 = max(10, args.steps // 2)
        log(f"[bench] FP64 companion: {k64} steps")
        r64 = run_gpu(pr, "f64", k64, args.warmup, autotune=not args.no_autotune)
        v64 = cells * k64 / (r64["event_ms"] * 1e-3)
        out["fp64"] = {"value": round(v64, 1), "ms_per_step": round(r64["event_ms"] / k64, 4),
                       "steps": k64, "tile": _tile(r64["tile_depth"]),
                       "roofline": roofline(r64["profile"], cells, "f64")}
    if not args.no_batch:
        log(f"[bench] batched workload: {args.batch_count} instances")
        try:
            out["batched"] = run_batch(count=args.batch_count, tile_depth=args.batch_tile_depth)
            log(f"[bench] batched: {out['batched']['value']:.3e} cell-updates/s")
        except Exception as e:  # the headline stands without it
            out["batched"] = {"error": repr(e)}
    if not args.no_serve:
        log(f"[bench] serving workload: {args.serve_count} requests")
        try:
            out["serving"] = run_serve(count=args.serve_count, rate=args.serve_rate)
            log(f"[bench] serving: p50 {out['serving']['p50_s']} s, p99 {out['serving']['p99_s']} s")
        except Exception as e:
            out["serving"] = {"error": repr(e)}
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
