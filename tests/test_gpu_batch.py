"""Batched advance: members of uneven sizes and kinds advanced by one launch per
stage (captured in a HIP graph) give exactly what each gives advanced alone, and
each stops at its own step target."""
import math

import numpy as np
import pytest

from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu, rel_l1
from helpers import oracle_sim

pytestmark = pytest.mark.gpu


def _members():
    return [
        (P.sod(40, transverse=6), 23),
        (P.sedov((16, 20, 12)), 17),
        (P.well_flow(16), 30),
        (P.cloud(20, seed=4), 11),
        (P.random_state((12, 9, 14), seed=8, potential=True,
                        bc=(P.OUTFLOW, P.OUTFLOW, P.REFLECT, P.REFLECT, P.PERIODIC, P.PERIODIC)), 25),
        (P.batch_instance(0, 3, steps=19), 19),
    ]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_equals_solo(dtype):
    need_gpu()
    from paper_1912_04855_amd.sim import Batch
    mem = _members()
    announce("batch_equals_solo", dtype, [m[0].shape for m in mem])
    solo = []
    for pr, steps in mem:
        s = gpu_sim(pr, dtype)
        assert s.advance(math.inf, steps) == steps
        solo.append((s.conserved(), s.time()))
        s.close()
    b = Batch(dtype)
    sims, slots = [], []
    for pr, steps in mem:
        s = gpu_sim(pr, dtype)
        sims.append(s)
        slots.append(b.add(s, steps))
    # uneven advances, including chunks past every member's target
    done = []
    for k in (4, 4, 7, 20):
        b.advance(k)
        done = b.poll()
    assert sorted(done) == sorted(slots)
    for q, s in enumerate(sims):
        b.remove(slots[q])
        U, t = s.conserved(), s.time()
        assert t[1] == mem[q][1]
        assert t == solo[q][1]
        assert np.array_equal(U, solo[q][0]), (q, rel_l1(U, solo[q][0]))
        s.close()
    b.close()


def test_batch_member_matches_oracle_fp64():
    need_gpu()
    from paper_1912_04855_amd.sim import Batch
    pr = P.sedov((16, 20, 12))
    o = oracle_sim(pr)
    for _ in range(15):
        o.step()
    announce("batch_vs_oracle")
    b = Batch("f64")
    other = gpu_sim(P.sod(32), "f64")
    s = gpu_sim(pr, "f64")
    b.add(other, 40)
    slot = b.add(s, 15)
    b.advance(10)
    b.advance(10)
    assert slot in b.poll()
    b.remove(slot)
    assert np.array_equal(s.conserved(), o.conserved())
    b.close()


def test_batch_admission_budget_and_slot_reuse():
    need_gpu()
    from paper_1912_04855_amd.sim import Batch, required_bytes
    announce("batch_budget")
    pr = P.sod(32)
    need = required_bytes(pr.shape, pr.h, dtype="f32")
    b = Batch("f32", budget_bytes=2 * need + need // 2)
    a, c = gpu_sim(pr, "f32"), gpu_sim(pr, "f32")
    d = gpu_sim(pr, "f32")
    sa = b.add(a, 5)
    b.add(c, 5)
    assert b.try_add(d, 5) is None          # over budget: waits
    b.advance(6)
    assert sa in b.poll()
    b.remove(sa)
    sd = b.try_add(d, 5)                    # memory freed: admitted, slot reused
    assert sd == sa
    b.advance(6)
    assert sorted(b.poll()) == sorted(b.members)
    b.close()


def test_member_cannot_be_changed_or_freed():
    """While a simulation belongs to a batch, the calls that would change or free
    it return CSPH_ERR_ARG before any work is issued; after removal they work."""
    need_gpu()
    import ctypes as C
    from paper_1912_04855_amd import _lib
    from paper_1912_04855_amd.sim import Batch
    L = _lib.load()
    pr = P.sod(16, transverse=4)
    announce("member_guard", pr.shape)
    s = gpu_sim(pr, "f32")
    b = Batch("f32")
    slot = b.add(s, 5)
    W = np.ascontiguousarray(pr.prim)
    h = s.handle
    inflow = (C.c_double * 5)(1.0, 0.0, 0.0, 0.0, 1.0)
    calls = {
        "destroy": lambda: L.csph_destroy(h),
        "set_stream": lambda: L.csph_set_stream(h, None),
        "set_state": lambda: L.csph_set_state(h, _lib.PRIMITIVE, W.ctypes.data),
        "set_potential": lambda: L.csph_set_potential(h, None),
        "set_boundary": lambda: L.csph_set_boundary(h, 0, _lib.OUTFLOW, inflow),
        "set_time": lambda: L.csph_set_time(h, 0.0, 0),
        "set_scheme": lambda: L.csph_set_scheme(h, _lib.LIM_MINMOD, _lib.FLUX_SWEPT_AV),
        "set_tile_depth": lambda: L.csph_set_tile_depth(h, 8),
        "step": lambda: L.csph_step(h, 0.0, None),
        "advance": lambda: L.csph_advance(h, math.inf, 1, None),
    }
    for name, fn in calls.items():
        assert fn() == _lib.ERR_ARG, name
    with pytest.raises(_lib.CsphError):
        s.close()
    # the member is untouched and still advances with the batch
    b.advance(5)
    assert b.poll() == [slot]
    assert s.time()[1] == 5
    b.remove(slot)
    assert L.csph_set_time(h, 0.0, 0) == _lib.OK
    s.close()
    b.close()
