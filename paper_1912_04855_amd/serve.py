"""Continuous-batching request loop for simulation jobs.

Requests (grid, problem kind, dtype, step count) arrive as a Poisson stream.
Each is admitted as soon as the device-memory budget allows, as a new member of
the running batch of its dtype: its state stays resident on the device, and it
advances together with whatever else is in flight (one launch per stage for the
whole batch, two batches -- FP32 and FP64 -- on two streams).  Finished members
are read back, removed and freed, which makes room for waiting requests.  Host
work per request (building the initial state, reading the result) runs on
worker threads so that it overlaps the device work of the others.
Latency is measured from arrival to the result being on the host.
"""
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import problems as P
from .sim import Batch, from_problem, required_bytes


@dataclass
class Record:
    rid: int
    kind: str
    dtype: str
    edge: int
    steps: int
    cells: int
    arrival: float
    admitted: float = 0.0     # initial state on the device, joined its batch
    done: float = 0.0         # last step finished on the device
    finished: float = 0.0     # result on the host
    state: Optional[np.ndarray] = None

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class ServeStats:
    records: List[Record] = field(default_factory=list)
    wall_s: float = 0.0
    peak_bytes: int = 0
    peak_members: int = 0

    def summary(self):
        lat = np.array([r.latency for r in self.records])
        work = sum(r.cells * r.steps for r in self.records)
        def mean(xs):
            return float(np.mean(xs)) if len(xs) else None

        return {
            "requests": len(self.records),
            # where the time goes, mean per request: building the initial state on the
            # device (from arrival), stepping in the batch, reading the result back
            "mean_build_s": mean([r.admitted - r.arrival for r in self.records]),
            "mean_device_s": mean([r.done - r.admitted for r in self.records]),
            "mean_readback_s": mean([r.finished - r.done for r in self.records]),
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p90_s": float(np.percentile(lat, 90)) if len(lat) else None,
            # with n requests the 99th percentile rests on the slowest n/100 of them
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_s": float(lat.mean()) if len(lat) else None,
            "cell_updates_per_s": work / self.wall_s if self.wall_s > 0 else None,
            "wall_s": self.wall_s,
            "peak_device_bytes": self.peak_bytes,
            "peak_members": self.peak_members,
        }


def _build(problem, req):
    """Initial state of one request on the device (runs on a worker thread)."""
    pr = problem(req)
    sim = from_problem(pr, dtype=req.dtype)
    return pr.cells, sim


def _read(sim, keep):
    """Result of a finished request to the host, then free it (worker thread)."""
    st = sim.conserved()
    sim.close()
    return st if keep else None


def serve(requests, budget_bytes=64 << 30, k_steps=8, keep_states=False, problem=None,
          clock=time.perf_counter, log=None, workers=4) -> ServeStats:
    """Run the request stream ``requests`` (``problems.Request``, arrival-ordered).

    The loop thread only admits, advances and polls.  Building a request's
    initial state on the device and reading a finished result back run on
    ``workers`` threads, so the GPU keeps advancing the batch meanwhile.  Device
    memory is reserved against the budget when a request is handed to a worker
    and released when its result has been read back."""
    from concurrent.futures import ThreadPoolExecutor

    problem = problem or P.serve_problem
    pending = sorted(requests, key=lambda r: r.arrival)
    batches: Dict[str, Batch] = {"f32": Batch("f32"), "f64": Batch("f64")}
    active: Dict[tuple, tuple] = {}  # (dtype, slot) -> (record, sim, bytes)
    building: List[tuple] = []       # (record, future, bytes), arrival order
    reading: List[tuple] = []        # (record, future, bytes)
    used = 0
    stats = ServeStats()
    pool = ThreadPoolExecutor(max_workers=workers)
    t0 = clock()
    qi = 0
    try:
        while qi < len(pending) or active or building or reading:
            now = clock() - t0
            # hand arrived requests to the workers while the memory budget allows
            while qi < len(pending) and pending[qi].arrival <= now:
                req = pending[qi]
                e = req.edge
                need = required_bytes((e, e, e), 1.0 / e, dtype=req.dtype)
                if used + need > budget_bytes and (active or building or reading):
                    break
                rec = Record(req.rid, req.kind, req.dtype, req.edge, req.steps, 0, req.arrival)
                building.append((rec, pool.submit(_build, problem, req), need))
                used += need
                stats.peak_bytes = max(stats.peak_bytes, used)
                qi += 1
            # members whose state is on the device join their batch, in arrival order
            while building and building[0][1].done():
                rec, fut, need = building.pop(0)
                rec.cells, sim = fut.result()
                slot = batches[rec.dtype].add(sim, rec.steps)
                rec.admitted = clock() - t0
                active[(rec.dtype, slot)] = (rec, sim, need)
                stats.peak_members = max(stats.peak_members, len(active))
            # results read back: the request is complete
            still = []
            for rec, fut, need in reading:
                if fut.done():
                    rec.state = fut.result()
                    rec.finished = clock() - t0
                    used -= need
                    stats.records.append(rec)
                    if log:
                        log(f"[serve] request {rec.rid} {rec.kind} {rec.edge}^3 {rec.dtype} "
                            f"{rec.steps} steps: {rec.latency * 1e3:.1f} ms")
                else:
                    still.append((rec, fut, need))
            reading = still
            if not active:
                time.sleep(0.002 if (building or reading) else
                           max(0.0, min(0.05, pending[qi].arrival - (clock() - t0)))
                           if qi < len(pending) else 0.002)
                continue
            # one graph replay of k steps per batch; the two batches run on their own
            # streams, so their work overlaps on the device
            for dt, b in batches.items():
                if any(key[0] == dt for key in active):
                    b.advance(k_steps)
            for dt, b in batches.items():
                if not any(key[0] == dt for key in active):
                    continue
                for slot in b.poll():
                    rec, sim, need = active.pop((dt, slot))
                    b.remove(slot)
                    rec.done = clock() - t0
                    reading.append((rec, pool.submit(_read, sim, keep_states), need))
    finally:
        pool.shutdown(wait=True)
        for b in batches.values():
            b.close()
    stats.wall_s = clock() - t0
    stats.records.sort(key=lambda r: r.rid)
    return stats


def solo(req: "P.Request", problem=None) -> np.ndarray:
    """The same request advanced alone (reference for the in-the-mix result)."""
    problem = problem or P.serve_problem
    s = from_problem(problem(req), dtype=req.dtype)
    s.advance(math.inf, req.steps)
    out = s.conserved()
    s.close()
    return out
