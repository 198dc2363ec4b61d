"""Tile-depth autotuner: the tile depths (one per stage sweep) change the
schedule, never the result; tuning a simulation or a batch leaves its state and
time untouched; the chosen depths are remembered for later simulations of the
same shape."""
import math

import numpy as np
import pytest

from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu

pytestmark = pytest.mark.gpu


def _problem():
    return P.random_state((20, 14, 33), seed=11, potential=True,
                          bc=(P.OUTFLOW, P.OUTFLOW, P.PERIODIC, P.PERIODIC, P.REFLECT, P.REFLECT))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tile_depth_changes_schedule_not_result(dtype):
    need_gpu()
    pr = _problem()
    ref = None
    # one depth for all stages, and mixed per-stage depths (stage P, C, E)
    for tz in (2, 4, 16, 64, (2, 64, 16), (64, 4, 2), (16, 2, 64)):
        announce("tile_depth", dtype, tz, pr.shape)
        s = gpu_sim(pr, dtype)
        s.tile_depth = tz
        assert s.tile_depth == (tuple(tz) if isinstance(tz, tuple) else (tz, tz, tz))
        assert s.advance(math.inf, 12) == 12
        U = s.conserved()
        # the FP64 totals of the last stage E cover exactly this depth's tiles
        tot = s.totals()
        h3 = pr.h ** 3
        for v in range(5):
            want = float(np.sum(U[v])) * h3
            assert abs(tot[v] - want) <= 1e-12 * max(1.0, float(np.sum(np.abs(U[v]))) * h3), (tz, v)
        if ref is None:
            ref = U
        else:
            assert np.array_equal(U, ref), tz
        s.close()


def test_tile_depth_rejects_bad_values():
    need_gpu()
    from paper_1912_04855_amd import _lib
    s = gpu_sim(P.sod(16), "f64")
    for bad in (0, 1, 65, -3, (2, 2, 65), (1, 8, 8)):
        with pytest.raises(_lib.CsphError):
            s.tile_depth = bad
    with pytest.raises(ValueError):
        s.tile_depth = (8, 8)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_autotune_leaves_sim_untouched_and_is_remembered(dtype):
    need_gpu()
    pr = _problem()
    announce("autotune", dtype, pr.shape)
    s = gpu_sim(pr, dtype)
    s.advance(math.inf, 3)
    U0, t0 = s.conserved(), s.time()
    tz, ms = s.autotune(trial_steps=2)
    assert len(tz) == 3 and all(d in (2, 4, 8, 16, 32, 64) for d in tz) and ms > 0
    assert s.tile_depth == tz
    assert s.time() == t0
    assert np.array_equal(s.conserved(), U0)
    s.advance(math.inf, 5)
    # a fresh simulation of the same shape starts from the tuned depth
    r = gpu_sim(pr, dtype)
    assert r.tile_depth == tz
    r.tile_depth = 2 if tz != (2, 2, 2) else 4
    r.advance(math.inf, 8)
    assert np.array_equal(s.conserved(), r.conserved())
    s.close()
    r.close()


def test_batch_autotune_restores_members():
    need_gpu()
    from paper_1912_04855_amd.sim import Batch
    mem = [(P.sod(40, transverse=6), 9), (P.sedov((16, 20, 12)), 7), (P.well_flow(16), 12)]
    announce("batch_autotune", [m[0].shape for m in mem])
    solo = []
    for pr, steps in mem:
        s = gpu_sim(pr, "f32")
        s.advance(math.inf, steps)
        solo.append(s.conserved())
        s.close()
    b = Batch("f32")
    sims, slots = [], []
    for pr, steps in mem:
        s = gpu_sim(pr, "f32")
        sims.append(s)
        slots.append(b.add(s, steps))
    b.advance(2)
    before = [(s.conserved(), s.time()) for s in sims]
    tz, ms = b.autotune(trial_steps=2)
    assert tz in (2, 4, 8, 16, 32, 64) and ms > 0
    for s, (U, t) in zip(sims, before):
        assert s.time() == t
        assert np.array_equal(s.conserved(), U)
        assert s.tile_depth == (tz, tz, tz)
    b.advance(20)
    assert sorted(b.poll()) == sorted(slots)
    for q, s in enumerate(sims):
        b.remove(slots[q])
        assert np.array_equal(s.conserved(), solo[q]), q
        s.close()
    b.close()
