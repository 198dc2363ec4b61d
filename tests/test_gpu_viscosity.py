"""Viscosity (the Sec. 4 extension) on the GPU against the oracle: the stage
fields of one step and 100 steps in FP64 (the same expressions in the same
order: to the last bit), the decaying shear wave in FP32, the viscous limit of
the time step, and a batch with viscous and inviscid members."""
import math

import numpy as np
import pytest

from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu, rel_l1, rel_l1_vars
from helpers import oracle_sim

pytestmark = pytest.mark.gpu

STAGES = ["msx", "msy", "msz", "Es", "xsx", "xsy", "xsz", "phis", "mtx", "mty", "mtz", "Et",
          "xtx", "xty", "xtz"]


def _viscous_mixed(nu=0.02):
    pr = P.random_state((12, 10, 9), seed=15, potential=True,
                        bc=(P.INFLOW, P.OUTFLOW, P.REFLECT, P.REFLECT, P.PERIODIC, P.PERIODIC))
    pr.inflow = {0: (1.1, 0.4, 0.05, -0.02, 0.9)}
    pr.nu = nu
    return pr


def _shear_wave(n=64, A=1e-3, nu=0.01):
    shape = (n, 4, 4)
    h = 1.0 / n
    x, _, _ = P.centres(shape, h)
    prim = np.zeros((5, 4, 4, n))
    prim[0] = 1.0
    prim[4] = 1.0
    prim[2] = np.broadcast_to(A * np.sin(2 * math.pi * x), prim.shape[1:])
    return P.Problem("shear_wave", shape, h, 1.4, 0.4, (P.PERIODIC,) * 6, prim, nu=nu)


def test_viscous_one_step_stages_fp64():
    need_gpu()
    pr = _viscous_mixed()
    o = oracle_sim(pr)
    dto = o.step()
    announce("viscous_one_step_fp64", pr.shape)
    g = gpu_sim(pr, "f64")
    assert g.step() == dto
    for f in STAGES:
        a, b = g.stage(f), o.field(f)
        scale = max(np.max(np.abs(b)), 1e-300)
        assert np.max(np.abs(a - b)) <= 1e-14 * scale, f
    assert rel_l1_vars(g.conserved(), o.conserved()) <= 1e-14
    g.close()


@pytest.mark.parametrize("name", ["mixed", "well_flow_24"])
def test_viscous_many_steps_fp64(name):
    need_gpu()
    if name == "mixed":
        pr = _viscous_mixed()
    else:
        pr = P.well_flow(24)
        pr.nu = 2e-3
    o = oracle_sim(pr)
    for _ in range(100):
        o.step()
    announce("viscous_many_steps_fp64", name, pr.shape)
    g = gpu_sim(pr, "f64")
    assert g.advance(math.inf, 100) == 100
    err = rel_l1_vars(g.conserved(), o.conserved())
    print(f"viscous {name}: FP64 relative L1 vs oracle after 100 steps = {err:.3e}")
    assert err <= 1e-12
    assert g.time()[0] == pytest.approx(o.time()[0], rel=1e-13)
    g.close()


def test_viscous_shear_wave_fp32():
    need_gpu()
    pr = _shear_wave()
    t_end = 0.5
    o = oracle_sim(pr)
    o.advance(t_end)
    announce("viscous_shear_fp32", pr.shape)
    g = gpu_sim(pr, "f32")
    g.advance(t_end)
    assert g.time()[0] == t_end
    Ug, Uo = g.conserved(), o.conserved()
    err = rel_l1(Ug, Uo)
    per = [rel_l1(Ug[v], Uo[v]) for v in (0, 2, 4)]
    n = pr.shape[0]
    xc = (np.arange(n) + 0.5) / n
    amp = 2 * np.mean((Ug[2] / Ug[0])[0, 0] * np.sin(2 * math.pi * xc))
    rate = -math.log(amp / 1e-3) / t_end
    exact = pr.nu * (2 * math.pi) ** 2
    print(f"shear wave FP32: relative L1 {err:.2e} (rho, m_y, E: "
          + ", ".join(f"{e:.1e}" for e in per) + f"); decay rate {rate:.5f} vs nu k^2 {exact:.5f}")
    assert err <= 1e-5 and max(per) <= 1e-5
    assert abs(rate - exact) <= 0.02 * exact
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_viscous_time_step_limit(dtype):
    need_gpu()
    pr = P.uniform_flow((8, 8, 8), u=(0.1, 0.0, 0.0))
    pr.nu = 10.0
    announce("viscous_dt", dtype)
    g = gpu_sim(pr, dtype)
    assert g.step() == 0.25 * pr.h ** 2 / pr.nu
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_with_viscous_member_equals_solo(dtype):
    need_gpu()
    from paper_1912_04855_amd.sim import Batch
    mem = [(_viscous_mixed(), 12), (P.sod(32), 15), (_shear_wave(32), 10)]
    announce("viscous_batch", dtype)
    solo = []
    for pr, steps in mem:
        s = gpu_sim(pr, dtype)
        assert s.advance(math.inf, steps) == steps
        solo.append(s.conserved())
        s.close()
    b = Batch(dtype)
    sims, slots = [], []
    for pr, steps in mem:
        s = gpu_sim(pr, dtype)
        sims.append(s)
        slots.append(b.add(s, steps))
    b.advance(20)
    assert sorted(b.poll()) == sorted(slots)
    for q, s in enumerate(sims):
        b.remove(slots[q])
        assert np.array_equal(s.conserved(), solo[q]), q
        s.close()
    b.close()
