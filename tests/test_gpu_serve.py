"""Continuous batching: requests admitted while others are in flight give the same
result as when run alone, bitwise (each member's arithmetic is independent of the
rest of the batch), under a memory budget that forces queueing."""
import numpy as np
import pytest

from paper_1912_04855_amd import problems as P

from gpu_common import announce, need_gpu

pytestmark = pytest.mark.gpu


def test_serve_results_equal_solo():
    need_gpu()
    from paper_1912_04855_amd import serve as S
    from paper_1912_04855_amd.sim import required_bytes
    reqs = P.serve_requests(count=14, rate=200.0, seed=3, edges=(12, 16, 20, 24), max_steps=40,
                            min_steps=5)
    announce("serve", [(r.kind, r.edge, r.dtype, r.steps) for r in reqs])
    # room for about three of the largest requests at once: later arrivals queue
    budget = 3 * required_bytes((24, 24, 24), 1 / 24, dtype="f64")
    stats = S.serve(reqs, budget_bytes=budget, k_steps=4, keep_states=True)
    assert len(stats.records) == len(reqs)
    assert stats.peak_bytes <= budget
    assert stats.peak_members >= 2
    for rec, req in zip(stats.records, reqs):
        assert rec.rid == req.rid
        ref = S.solo(req)
        assert np.array_equal(rec.state, ref), (req.kind, req.edge, req.dtype)
    summ = stats.summary()
    print("serve summary:", summ)
    assert summ["p99_s"] >= summ["p50_s"] > 0
