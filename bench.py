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

import numpy as np

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

# Algorithmic bytes per interior cell of each stage kernel, in words (4 B in
# FP32, 8 B in FP64): every input of the kernel read once, every output written
# once.  The FP32 build does not store the particle offsets xi*, xi^{n+1}: it
# forms them from the momenta where they are needed.
#   stage P: read U^n (5) + psi (1);  write m*, E* (4) + psi(r*) (1) + phi* (1)
#            [FP64 also writes xi* (3)]
#   stage C: read rho, m* (4) + phi* (1) + psi(r*) (1) + m^n, E^n (4) + E* (1);
#            write m~, E~ (4)  [FP64 reads xi* (3) and writes xi^{n+1} (3)]
#   stage E: read U^n (5) + m~, E~ (4) + m* (3) [FP64: xi^{n+1} (3)];  write U^{n+1} (5)
RW = {"f32": {"stage_p": (6, 6), "stage_c": (11, 4), "stage_e": (12, 5)},
      "f64": {"stage_p": (6, 9), "stage_c": (14, 7), "stage_e": (12, 5)}}
WORDS = {t: {k: r + w for k, (r, w) in m.items()} for t, m in RW.items()}
# Algorithmic floating-point operations per interior cell of each stage (each
# +, -, *, /, sqrt, min, max counted once; a fused multiply-add is two), as the
# method defines them, not as the kernels happen to issue them:
#   stage P: primitives (14) + the 13 lattice pair terms of A (119), D[psi] (54)
#            and B (212) + rho u.D[psi] (7) + the predictor update (20) + psi at
#            r* (27) + the lattice divergence of u^n (27 pair components x 3 = 81)
#            + the predicted volume and phi* (5)                          = 539
#   stage C: u* = m*/rho (3) + the same lattice sums on the predicted particles
#            (119 + 54 + 212 + 7 = 392) + the corrector update (16)        = 411
#   stage E: three faces per cell (a face is shared by two cells) x 154 (slopes
#            and minmod 45, reconstruction and swept flux 41, the swept width at
#            the foot of the face's trajectory 6, acoustic damping 62) + the
#            update (35) + the next step's signal speed (21) and the totals (5) = 523
FLOPS = {"stage_p": 539, "stage_c": 411, "stage_e": 523}
# What bounds each kernel is read from rocprofv3 counters of the current kernel
# source (profiles/traffic.json): the share of the launch in which the SIMDs
# issue vector-ALU instructions, SQ_ACTIVE_INST_VALU / (CU count x GRBM_GUI_ACTIVE)
# (AMD's VALUBusy).  A kernel busier than VALU_BOUND is reported against the
# vector-ALU peak, any other against HBM.  Without a summary of the current
# source the last measured bounds below stand.
VALU_BOUND = 0.75
BOUND_MEASURED = {"stage_p": "alu", "stage_c": "hbm", "stage_e": "hbm"}
KERNEL_NAMES = {"stage_p": "k_stage_p", "stage_c": "k_stage_c", "stage_e": "k_stage_e"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _depths(text):
    """--tile-depth: one depth for every stage, or 'p,c,e'."""
    v = [int(x) for x in str(text).split(",")]
    if len(v) not in (1, 3):
        raise argparse.ArgumentTypeError("one depth or three (stage P, C, E)")
    return v[0] if len(v) == 1 else tuple(v)


def _tile(depths, dtype="f32"):
    """Tile shapes and the z-depth of each stage's sweep (single grid: FP32 stages
    P and C take 64x4 tiles, FP64 and stage E 32x8)."""
    shapes = "P/C 64x4, E 32x8" if dtype == "f32" else "32x8"
    return shapes + ", z-depth P/C/E " + "/".join(str(d) for d in depths)


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


def run_large(n=1024, steps=10, warmup=2, tile_depth=0):
    """The potential-well flow on an n^3 FP32 grid (1024^3: about 91 GB of HBM),
    set up without a host copy of the state: every cell is filled with the
    inflow state on the device, the potential is uploaded; events around
    `steps` steps (autotuning would need a second grid, so the tile depths are
    the ones given)."""
    import torch
    from paper_1912_04855_amd import problems as P
    from paper_1912_04855_amd.sim import Sim

    pr = P.well_flow(8)  # the workload's constants (state, boundaries)
    state = np.array(pr.inflow[0], dtype=np.float64)
    sim = Sim((n, n, n), 1.0 / n, gamma=pr.gamma, cfl=pr.cfl, rho_vac=pr.rho_vac, dtype="f32",
              torch=True)
    for f in range(6):
        sim.set_boundary(f, pr.bc[f], state if pr.bc[f] == P.INFLOW else None)
    sim.fill_state(state)
    psi = P.gaussian_well((n, n, n), 1.0 / n)
    sim.set_potential(psi)
    del psi
    if tile_depth:
        sim.tile_depth = tile_depth
    stream = torch.cuda.current_stream()
    sim.advance(math.inf, warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    k = sim.advance(math.inf, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    assert k == steps, (k, steps)
    ms = ev0.elapsed_time(ev1)
    tz = sim.tile_depth
    sim.close()
    return {"value": round(n ** 3 * steps / (ms * 1e-3), 1), "unit": "cell-updates/s",
            "ms_per_step": round(ms / steps, 4), "steps": steps, "cells": n ** 3, "dtype": "f32",
            "tile": _tile(tz),
            "workload": f"potential-well flow {n}^3 (the headline workload's state, potential "
                        "and boundaries on a 64x larger grid; state filled on the device)"}


def run_share(n=256, gpus=8, steps=100, warmup=5):
    """One GPU's share of the n^3 potential-well flow split into `gpus` z-slabs:
    n/gpus owned planes plus 3 overlap planes on either side (one step reads
    U^n at most 3 cells away, so the owned planes advance exactly as in the
    whole grid), z faces OUTFLOW standing in for the halo.  Only the owned cells
    count as cell-updates; the overlap planes are the redundant halo compute."""
    from paper_1912_04855_amd import problems as P
    planes, overlap = n // gpus, 3
    pr = P.z_slab(P.well_flow(n), 0, planes, overlap)
    r = run_gpu(pr, "f32", steps, warmup)  # its own tile depths: 38 planes, not 256
    owned = n * n * planes
    halo = 2 * overlap * 5 * n * n * 4  # U^n planes received per step (both neighbours), FP32
    return {"value": round(owned * steps / (r["event_ms"] * 1e-3), 1), "unit": "cell-updates/s",
            "ms_per_step": round(r["event_ms"] / steps, 4), "steps": steps, "shape": list(pr.shape),
            "owned_cells": owned, "dtype": "f32", "tile": _tile(r["tile_depth"]),
            "halo_bytes_per_step": halo,
            "kernels_ms": {k: round(v[0], 5) for k, v in r["profile"].items()},
            "workload": f"one GPU's share of the potential-well flow {n}^3 in {gpus} z-slabs: "
                        f"{planes} owned planes + {overlap} overlap planes each side "
                        f"({n}x{n}x{planes + 2 * overlap}); the halo exchange itself is not run"}


def run_gravity(n=256, steps=50, warmup=3, tile_depth=0, boxes=("periodic", "isolated")):
    """The self-gravity extension on an n^3 FP32 grid: the seeded smooth state
    (rho, p in [0.7, 1.3], |u| <= 0.3, a smooth external potential) with G = 1,
    once on a periodic box (spectral solve of the discrete Poisson equation) and
    once with every face OUTFLOW (the free-space potential through the box
    zero-padded to 2n per axis).  Per box: time per step and the self-gravity
    group's time (the Poisson solve and the ghosts of its two potentials)."""
    from paper_1912_04855_amd import problems as P
    out = {}
    for name, bc in (("periodic", None), ("isolated", (P.OUTFLOW,) * 6)):
        if name not in boxes:
            continue
        pr = P.smooth_state((n, n, n), seed=3, bc=bc)
        pr.grav = 1.0
        r = run_gpu(pr, "f32", steps, warmup, autotune=False, tile_depth=tile_depth)
        out[name] = {"value": round(pr.cells * steps / (r["event_ms"] * 1e-3), 1), "unit": "cell-updates/s",
                     "ms_per_step": round(r["event_ms"] / steps, 4), "steps": steps,
                     "self_gravity_ms": round(r["profile"]["self_gravity"][0], 4),
                     "kernels_ms": {k: round(v[0], 5) for k, v in r["profile"].items()}}
    out["workload"] = (f"self-gravitating smooth state {n}^3 FP32, G = 1: periodic box and isolated "
                       "box (every face OUTFLOW)")
    return out


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


def bounds(dtype, cells):
    """Each stage kernel's bound and measured VALU-busy share (None without a
    counter summary of the current source)."""
    out = {}
    for k in WORDS[dtype]:
        rec = _counters(KERNEL_NAMES[k], dtype, cells)
        busy = rec.get("valu_busy") if rec else None
        if busy is None:
            out[k] = (BOUND_MEASURED[k], None)
        else:
            out[k] = ("alu" if busy >= VALU_BOUND else "hbm", busy)
    return out


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
    bd = bounds(dtype, cells)
    per = {k: {"avg_ms": round(prof[k][0], 5), "launches": prof[k][1], "bound": bd[k][0],
               "valu_busy": bd[k][1],
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
    main = hbm if bd[dom][0] == "hbm" else alu
    out = {"bound": bd[dom][0], "kernel": KERNEL_NAMES[dom], "achieved": main["achieved"],
           "peak": main["peak"], "unit": main["unit"], "frac": main["frac"], "traffic": traffic,
           "alu": alu, "hbm": hbm, "kernels": per,
           # the step's other launches: three ghost fills (the first timed with the
           # step's opening launch) and the closing bookkeeping launch
           "other_kernels": {k: {"avg_ms": round(prof[k][0], 5), "launches": prof[k][1]}
                             for k in ("ghost_fill", "bookkeeping") if k in prof}}
    if bd[dom][1] is not None:
        out["valu_busy"] = bd[dom][1]
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


KERNEL_SOURCES = ("csph_gravity.hip", "csph_internal.h", "csph_kernels.hip")


def source_hash():
    """Hash of the kernel sources (the device code and the structures it shares
    with the host; not the host runtime) with comments and blank space removed,
    so that a counter summary stays tied to the kernels, not to their prose."""
    import hashlib
    import re
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1912_04855_amd", "csrc")
    for f in KERNEL_SOURCES:
        txt = open(os.path.join(d, f), encoding="utf-8").read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", " ", txt)
        h.update(" ".join(txt.split()).encode())
    return h.hexdigest()[:16]


def host_description():
    """CPU model, cores and threads of this host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    d = {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
                "Thread(s) per core": "threads_per_core"}
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                d[keys[k.strip()]] = v.strip()
    except Exception:
        pass
    if "model" not in d:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    d["model"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return d


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
                      f"single-threaded C oracle, {el:.1f} s",
            "host": host_description()}


def _oracle_batch_member(args):
    """One batch instance stepped by the oracle (a worker process of cpu_box)."""
    master, k, steps = args
    import oracle as O
    from paper_1912_04855_amd import problems as P
    pr = P.batch_instance(master, k, steps=steps)
    s = O.OracleSim(pr.shape, pr.h, gamma=pr.gamma, cfl=pr.cfl, rho_vac=pr.rho_vac, bc=pr.bc,
                    inflow=pr.inflow_list())
    s.set_primitive(pr.prim)
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step()
    return pr.cells * steps, time.perf_counter() - t0


def cpu_box(instances=32, steps=4, master=0, batch_count=512, batch_steps=100):
    """The multi-instance comparator of the batched workload: one oracle process
    per host core (at most 16, the CPU share that comes with one GPU) on the first
    `instances` members of the batch, `steps` steps each; the aggregate rate is
    extrapolated to the whole batch (batch_count members, batch_steps steps)."""
    import multiprocessing as mp
    from paper_1912_04855_amd import problems as P
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")  # fresh interpreters: nothing of this process's GPU state
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_batch_member, [(master, k, steps) for k in range(instances)],
                       chunksize=1)
    wall = time.perf_counter() - t0
    work = sum(r[0] for r in res)
    # each process's own stepping rate, measured while all of them run at once
    # (shared caches and memory bandwidth included), times the processes
    rate = workers * work / sum(r[1] for r in res)
    total = sum(int(np.prod(P.batch_shape(master, k)[0])) for k in range(batch_count)) * batch_steps
    return {"value": round(rate, 1), "unit": "cell-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"{instances} of the {batch_count} batch members, {steps} FP64 steps each, "
                      f"one single-threaded oracle process per core ({wall:.1f} s wall with "
                      f"process start-up); value = processes x their mean stepping rate",
            "wall_rate": round(work / wall, 1),
            "extrapolated_batch_s": round(total / rate, 1)}


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
    ap.add_argument("--serve-count", type=int, default=80)
    ap.add_argument("--serve-rate", type=float, default=1.2,
                    help="mean arrival rate of the serving workload (requests per second)")
    ap.add_argument("--no-cloud", action="store_true", help="skip the gas-vacuum cloud workload")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 well-flow workload")
    ap.add_argument("--no-gravity", action="store_true",
                    help="skip the self-gravity workload (periodic and isolated boxes)")
    ap.add_argument("--gravity-only", action="store_true",
                    help="only the self-gravity workload, --steps steps (for profiling)")
    ap.add_argument("--gravity-box", default="both", choices=["both", "periodic", "isolated"])
    ap.add_argument("--no-share", action="store_true",
                    help="skip one GPU's z-slab share of the well flow (8 slabs)")
    ap.add_argument("--cloud-steps", type=int, default=50)
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
    if args.gravity_only:
        boxes = ("periodic", "isolated") if args.gravity_box == "both" else (args.gravity_box,)
        r = run_gravity(args.n, args.steps, args.warmup, tile_depth=args.tile_depth, boxes=boxes)
        print(json.dumps({"gravity": r}), flush=True)
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
    out = {
        "metric": "cell-updates/s", "value": round(value, 1), "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"potential-well flow {args.n}^3 (Mach-2 inflow, "
                               f"psi=-exp(-r^2/0.01), gamma=5/3)",
                   "cells": cells, "dtype": args.dtype, "parallelism": "single GPU",
                   "tile": _tile(r["tile_depth"], args.dtype)},
        "roofline": rl,
        "algorithmic_hbm_frac": round(value * (44 if args.dtype == "f32" else 88) / HBM_PEAK, 4),
    }
    if not args.no_fp64 and args.dtype == "f32":
        k64 = max(10, args.steps // 2)
        log(f"[bench] FP64 companion: {k64} steps")
        r64 = run_gpu(pr, "f64", k64, args.warmup, autotune=not args.no_autotune)
        v64 = cells * k64 / (r64["event_ms"] * 1e-3)
        out["fp64"] = {"value": round(v64, 1), "ms_per_step": round(r64["event_ms"] / k64, 4),
                       "steps": k64, "tile": _tile(r64["tile_depth"], "f64"),
                       "roofline": roofline(r64["profile"], cells, "f64")}
    if not args.no_cloud:
        log(f"[bench] gas-vacuum cloud 384^3 f32: {args.cloud_steps} steps")
        try:
            prc = P.cloud(384)
            rc = run_gpu(prc, "f32", args.cloud_steps, args.warmup, autotune=not args.no_autotune)
            vc = prc.cells * args.cloud_steps / (rc["event_ms"] * 1e-3)
            out["cloud"] = {"value": round(vc, 1), "unit": "cell-updates/s",
                            "ms_per_step": round(rc["event_ms"] / args.cloud_steps, 4),
                            "steps": args.cloud_steps, "cells": prc.cells, "dtype": "f32",
                            "tile": _tile(rc["tile_depth"]),
                            "kernels_ms": {k: round(v[0], 5) for k, v in rc["profile"].items()},
                            "workload": "gas-vacuum cloud 384^3 (rho = 1 - r^2/0.09 with 1% "
                                        "SplitMix64 noise, Plummer psi, vacuum outside, "
                                        "gamma = 5/3, outflow faces)"}
            log(f"[bench] cloud: {vc:.3e} cell-updates/s")
            del prc
        except Exception as e:
            out["cloud"] = {"error": repr(e)}
    if not args.no_gravity:
        log(f"[bench] self-gravity {args.n}^3 f32: periodic and isolated boxes")
        try:
            out["gravity"] = run_gravity(args.n, 50, 3, tile_depth=r["tile_depth"])
            log(f"[bench] gravity: periodic {out['gravity']['periodic']['ms_per_step']} ms/step, "
                f"isolated {out['gravity']['isolated']['ms_per_step']} ms/step")
        except Exception as e:
            out["gravity"] = {"error": repr(e)}
    if not args.no_share:
        log(f"[bench] one GPU's z-slab share of the {args.n}^3 well flow (8 slabs)")
        try:
            out["share"] = run_share(args.n, 8, args.steps, args.warmup)
            log(f"[bench] share: {out['share']['value']:.3e} owned cell-updates/s")
        except Exception as e:
            out["share"] = {"error": repr(e)}
    if not args.no_large:
        log("[bench] potential-well flow 1024^3 f32: 10 steps")
        try:
            out["large"] = run_large(1024, 10, tile_depth=r["tile_depth"])
            log(f"[bench] large: {out['large']['value']:.3e} cell-updates/s")
        except Exception as e:
            out["large"] = {"error": repr(e)}
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
        if not args.no_batch:
            log("[bench] CPU box comparator of the batched workload")
            try:
                out["cpu_box_batched"] = cpu_box(batch_count=args.batch_count)
            except Exception as e:
                out["cpu_box_batched"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
