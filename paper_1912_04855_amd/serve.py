"""Continuous-batching request loop for simulation jobs.

Requests (grid, problem kind, dtype, step count) arrive as a Poisson stream.
Each is admitted as soon as the device-memory budget allows, as a new member of
the running batch of its dtype: its state stays resident on the device, and it
advances together with whatever else is in flight (one launch per stage for the
whole batch, two batches -- FP32 and FP64 -- on two streams).  Finished members
are read back, removed and freed, which makes room for waiting requests.
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
    admitted: float = 0.0
    finished: float = 0.0
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
        return {
            "requests": len(self.records),
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_s": float(lat.mean()) if len(lat) else None,
            "cell_updates_per_s": work / self.wall_s if self.wall_s > 0 else None,
            "wall_s": self.wall_s,
            "peak_device_bytes": self.peak_bytes,
            "peak_members": self.peak_members,
        }


def serve(requests, budget_bytes=64 << 30, k_steps=8, keep_states=False, problem=None,
          clock=time.perf_counter, log=None) -> ServeStats:
    """Run the request stream ``requests`` (``problems.Request``, arrival-ordered)."""
    problem = problem or P.serve_problem
    pending = sorted(requests, key=lambda r: r.arrival)
    batches: Dict[str, Batch] = {"f32": Batch("f32"), "f64": Batch("f64")}
    active: Dict[tuple, tuple] = {}  # (dtype, slot) -> (record, sim, bytes)
    used = 0
    stats = ServeStats()
    t0 = clock()
    qi = 0
    try:
        while qi < len(pending) or active:
            now = clock() - t0
            # admit every arrived request the memory budget allows, in arrival order
            while qi < len(pending) and pending[qi].arrival <= now:
                req = pending[qi]
                pr = problem(req)
                need = required_bytes(pr.shape, pr.h, dtype=req.dtype, gamma=pr.gamma,
                                      cfl=pr.cfl, rho_vac=pr.rho_vac)
                if used + need > budget_bytes and active:
                    break
                sim = from_problem(pr, dtype=req.dtype)
                slot = batches[req.dtype].add(sim, req.steps)
                rec = Record(req.rid, req.kind, req.dtype, req.edge, req.steps, pr.cells,
                             req.arrival, admitted=clock() - t0)
                active[(req.dtype, slot)] = (rec, sim, need)
                used += need
                stats.peak_bytes = max(stats.peak_bytes, used)
                stats.peak_members = max(stats.peak_members, len(active))
                qi += 1
            if not active:
                if qi < len(pending):
                    time.sleep(max(0.0, min(0.05, pending[qi].arrival - (clock() - t0))))
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
                    st = sim.conserved()
                    rec.finished = clock() - t0
                    if keep_states:
                        rec.state = st
                    sim.close()
                    used -= need
                    stats.records.append(rec)
                    if log:
                        log(f"[serve] request {rec.rid} {rec.kind} {rec.edge}^3 {rec.dtype} "
                            f"{rec.steps} steps: {rec.latency * 1e3:.1f} ms")
    finally:
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
