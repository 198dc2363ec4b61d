"""Sources and sinks (the Sec. 4 extension) on the GPU against the oracle: the
FP64 build applies the same per-cell operations in the same order, half before
the hydrodynamic step and half inside stage E's update, so its stage fields and
states follow the oracle to rounding of the order of the last bit; FP32 against
closed forms and the oracle; a 256^3 mass budget; refusals."""
import math

import numpy as np
import pytest

from paper_1912_04855_amd import _lib
from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu, rel_l1, rel_l1_vars
from helpers import oracle_sim

pytestmark = pytest.mark.gpu

STAGES = ["msx", "msy", "msz", "Es", "xsx", "xsy", "xsz", "phis", "mtx", "mty", "mtz", "Et",
          "xtx", "xty", "xtz"]


def _rates(shape_zyx, seed):
    """Seeded rates: two cells in three sources in [0, 2], one in three sinks in [-3, 0]."""
    n = int(np.prod(shape_zyx))
    r = P.uniform01(seed, np.arange(n, dtype=np.uint64)).reshape(shape_zyx)
    q = 2.0 * r
    q[r > 2.0 / 3.0] = -9.0 * (r[r > 2.0 / 3.0] - 2.0 / 3.0)
    return q


def _mixed(seed=31):
    pr = P.random_state((12, 10, 9), seed=seed, potential=True,
                        bc=(P.INFLOW, P.OUTFLOW, P.REFLECT, P.REFLECT, P.PERIODIC, P.PERIODIC))
    pr.inflow = {0: (1.1, 0.4, 0.05, -0.02, 0.9)}
    pr.src = _rates((9, 10, 12), seed + 1)
    pr.eps_src = 0.7
    return pr


def test_sources_one_step_stages_fp64():
    need_gpu()
    pr = _mixed()
    o = oracle_sim(pr)
    dto = o.step()
    announce("sources_one_step_fp64", pr.shape)
    g = gpu_sim(pr, "f64")
    assert g.step() == dto
    for f in STAGES:
        a, b = g.stage(f), o.field(f)
        scale = max(np.max(np.abs(b)), 1e-300)
        assert np.max(np.abs(a - b)) <= 1e-14 * scale, f
    assert rel_l1_vars(g.conserved(), o.conserved()) <= 1e-14
    g.close()


@pytest.mark.parametrize("name", ["mixed", "gravity"])
def test_sources_many_steps_fp64(name):
    need_gpu()
    if name == "mixed":
        pr, steps = _mixed(), 100
    else:
        # with self-gravity: the first half of the source precedes the Poisson solve
        pr = P.random_state((16, 8, 8), seed=8, potential=True)
        pr.grav = 0.6
        pr.src = _rates((8, 8, 16), 9)
        pr.eps_src = 1.2
        steps = 40
    o = oracle_sim(pr)
    for _ in range(steps):
        o.step()
    announce("sources_many_steps_fp64", name)
    g = gpu_sim(pr, "f64")
    assert g.advance(math.inf, steps) == steps
    err = rel_l1_vars(g.conserved(), o.conserved())
    print(f"sources {name}: FP64 relative L1 vs oracle after {steps} steps = {err:.3e}")
    assert err <= (1e-12 if name == "mixed" else 1e-10)
    g.close()


def test_changing_and_clearing_sources_fp64():
    need_gpu()
    pr = _mixed(41)
    o = oracle_sim(pr)
    announce("sources_change_fp64")
    g = gpu_sim(pr, "f64")
    q2 = -0.5 * _rates((9, 10, 12), 43)
    for s in (o, g):
        for _ in range(5):
            s.step()
        s.set_source(q2, 0.3)
        for _ in range(5):
            s.step()
        s.set_source(None)
        for _ in range(5):
            s.step()
    assert rel_l1_vars(g.conserved(), o.conserved()) <= 1e-13
    g.close()


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.1)])
def test_uniform_source_fp32(u):
    need_gpu()
    pr = P.uniform_flow((16, 8, 8), u=u)
    pr.src = np.full((8, 8, 16), 0.5)
    pr.eps_src = 2.0
    announce("uniform_source_fp32", u)
    g = gpu_sim(pr, "f32")
    U0 = g.conserved()
    g.advance(0.3)
    t = g.time()[0]
    U = g.conserved()
    # FP32 rounding of ~15 steps
    assert np.max(np.abs(U[0] - (1.0 + 0.5 * t))) <= 5e-6
    assert np.max(np.abs(U[1:4] - U0[1:4])) <= 5e-6
    assert np.max(np.abs(U[4] - (U0[4] + 0.5 * 2.0 * t))) <= 1e-5
    g.close()


def test_source_pair_fp32():
    need_gpu()
    n = 128
    shape = (n, 4, 4)
    x, _, _ = P.centres(shape, 1.0 / n)
    prim = np.zeros((5, 4, 4, n))
    prim[0] = 1.0
    prim[4] = 1.0
    pr = P.Problem("source_pair", shape, 1.0 / n, 1.4, 0.4, (P.PERIODIC,) * 6, prim, t_end=0.2)
    q = 2.0 * np.exp(-(x - 0.5) ** 2 / 0.01) - np.exp(-(x - 0.2) ** 2 / 0.005)
    pr.src = np.ascontiguousarray(np.broadcast_to(q, (4, 4, n)))
    pr.eps_src = 1.5
    o = oracle_sim(pr)
    o.advance(pr.t_end)
    announce("source_pair_fp32")
    g = gpu_sim(pr, "f32")
    g.advance(pr.t_end)
    err = rel_l1(g.conserved(), o.conserved())
    print(f"source pair FP32: relative L1 vs oracle {err:.2e}")
    assert err <= 1e-5
    g.close()


def test_mass_budget_at_size():
    # the benchmark's grid: a periodic gas with a seeded positive rate field gains
    # exactly sum(q) h^3 t of mass (FP64 totals of the FP32 state)
    need_gpu()
    n = 256
    pr = P.smooth_state((n, n, n), seed=4, potential=False)
    pr.src = 0.5 * P.uniform01(7, np.arange(n ** 3, dtype=np.uint64)).reshape(n, n, n)
    pr.eps_src = 1.0
    announce("source_mass_budget", n)
    g = gpu_sim(pr, "f32")
    m0 = g.totals()[0]
    assert g.advance(math.inf, 5) == 5
    t = g.time()[0]
    m1 = g.totals()[0]
    expect = m0 + pr.src.astype(np.float32).astype(np.float64).sum() * pr.h ** 3 * t
    print(f"mass budget 256^3 FP32: {m1:.9f} vs {expect:.9f}")
    assert abs(m1 - expect) <= 2e-6 * expect
    g.close()


def test_source_refusals():
    need_gpu()
    from paper_1912_04855_amd.sim import Batch, Sim
    announce("source_refusals")
    pr = P.uniform_flow((16, 8, 8))
    g = gpu_sim(pr, "f32")
    with pytest.raises(_lib.CsphError):
        g.set_source(np.full((8, 8, 16), np.nan), 1.0)
    with pytest.raises(_lib.CsphError):
        g.set_source(1.0, -1.0)
    g.set_source(1.0, 1.0)
    b = Batch("f32")
    with pytest.raises(_lib.CsphError):
        b.add(g, 3)
    g.set_source(None)
    slot = b.add(g, 3)
    b.advance(3)
    b.remove(slot)
    b.close()
    g.close()
    s = Sim((16, 8, 8), 1.0 / 16, dtype="f32", static=True)
    with pytest.raises(_lib.CsphError):
        s.set_source(1.0, 1.0)
    s.close()


@pytest.mark.parametrize("box", ["periodic", "isolated"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_all_extensions_together(dtype, box):
    # viscosity, self-gravity and sources and sinks on one grid with an external
    # potential, against the oracle: a periodic box, and an isolated one (every
    # face OUTFLOW, the free-space potential)
    need_gpu()
    pr = P.random_state((16, 12, 8), seed=17, potential=True,
                        bc=(P.OUTFLOW,) * 6 if box == "isolated" else None)
    pr.nu = 0.01
    pr.grav = 0.4
    pr.src = _rates((8, 12, 16), 18)
    pr.eps_src = 0.9
    o = oracle_sim(pr)
    for _ in range(30):
        o.step()
    announce("all_extensions", dtype, box)
    g = gpu_sim(pr, dtype)
    assert g.advance(math.inf, 30) == 30
    err = rel_l1_vars(g.conserved(), o.conserved())
    print(f"viscosity + gravity + sources {dtype} {box}: relative L1 vs oracle after 30 steps = {err:.3e}")
    assert err <= (1e-11 if dtype == "f64" else 2e-5)
    assert g.time()[0] == pytest.approx(o.time()[0], rel=1e-12 if dtype == "f64" else 1e-5)
    g.close()
