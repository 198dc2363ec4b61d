"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: FP64 build within 1e-12 relative L1 after 100 steps (it evaluates the
same expressions in the same order, so the cases agree to the last bit); FP32
build within 1e-5 relative L1 (of the whole conserved state, and of density,
momentum and energy each) on smooth flows, and shock positions within one cell.  Each stage's output is also compared after one step, so a failure names
the stage.
"""
import math

import numpy as np
import pytest

from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu, rel_l1, rel_l1_vars
from helpers import oracle_sim

pytestmark = pytest.mark.gpu

STAGES = ["msx", "msy", "msz", "Es", "xsx", "xsy", "xsz", "phis", "mtx", "mty", "mtz", "Et",
          "xtx", "xty", "xtz"]


def _mixed_bc_problem():
    pr = P.random_state((12, 10, 9), seed=5, potential=True,
                        bc=(P.INFLOW, P.OUTFLOW, P.REFLECT, P.REFLECT, P.PERIODIC, P.PERIODIC))
    pr.inflow = {0: (1.1, 0.4, 0.05, -0.02, 0.9)}
    return pr


CASES_ONE_STEP = {
    "mixed_bc": _mixed_bc_problem,
    "well_flow_16": lambda: P.well_flow(16),
    "cloud_16": lambda: P.cloud(16, seed=2),
    "sedov_12x14x16": lambda: P.sedov((12, 14, 16)),
    "sod_x": lambda: P.sod(32),
    "sod_z": lambda: P.sod(32, axis=2),
}


@pytest.mark.parametrize("name", list(CASES_ONE_STEP))
def test_one_step_stages_fp64(name):
    need_gpu()
    pr = CASES_ONE_STEP[name]()
    o = oracle_sim(pr)
    dto = o.step()
    announce("one_step_stages_fp64", name, pr.shape)
    g = gpu_sim(pr, "f64")
    dtg = g.step()
    assert dtg == dto
    for f in STAGES:
        a, b = g.stage(f), o.field(f)
        scale = max(np.max(np.abs(b)), 1e-300)
        assert np.max(np.abs(a - b)) <= 1e-14 * scale, f
    Ug, Uo = g.conserved(), o.conserved()
    assert rel_l1_vars(Ug, Uo) <= 1e-14
    g.close()


@pytest.mark.parametrize("name,steps", [("sod", None), ("well_flow_24", 100), ("cloud_20", 100),
                                        ("sedov_16", 100), ("mixed_bc", 100)])
def test_many_steps_fp64(name, steps):
    need_gpu()
    pr = {"sod": lambda: P.sod(128), "well_flow_24": lambda: P.well_flow(24),
          "cloud_20": lambda: P.cloud(20, seed=1), "sedov_16": lambda: P.sedov((16, 16, 16)),
          "mixed_bc": _mixed_bc_problem}[name]()
    o = oracle_sim(pr)
    announce("many_steps_fp64", name, pr.shape, steps)
    g = gpu_sim(pr, "f64")
    if steps is None:
        no = o.advance(pr.t_end)
        ng = g.advance(pr.t_end)
        assert no == ng
        assert g.time()[0] == o.time()[0] == pr.t_end
    else:
        for _ in range(steps):
            o.step()
        assert g.advance(math.inf, steps) == steps
        assert g.time()[0] == pytest.approx(o.time()[0], rel=1e-13)
    err = rel_l1_vars(g.conserved(), o.conserved())
    print(f"{name}: FP64 relative L1 vs oracle = {err:.3e}")
    assert err <= 1e-12
    tg, to = g.totals(), o.totals()
    np.testing.assert_allclose(tg, to, rtol=1e-12, atol=1e-14 * np.max(np.abs(to)))
    g.close()


@pytest.mark.parametrize("name,steps,tol", [("well_flow_24", 50, 1e-5),
                                            ("acoustic_64", 100, 1e-6),
                                            ("advected_64", 100, 1e-5)])
def test_smooth_flows_fp32(name, steps, tol):
    need_gpu()
    pr = {"well_flow_24": lambda: P.well_flow(24),
          "acoustic_64": lambda: P.acoustic_wave(64, eps=1e-3),
          "advected_64": lambda: P.advected_density(64)}[name]()
    o = oracle_sim(pr)
    for _ in range(steps):
        o.step()
    announce("smooth_fp32", name, pr.shape, steps)
    g = gpu_sim(pr, "f32")
    g.advance(math.inf, steps)
    Ug, Uo = g.conserved(), o.conserved()
    err = rel_l1(Ug, Uo)
    per = [rel_l1(Ug[v], Uo[v]) for v in range(5)]
    mom = rel_l1(Ug[1:4], Uo[1:4])
    print(f"{name}: FP32 relative L1 of the state vs FP64 oracle = {err:.3e} (per variable "
          + ", ".join(f"{e:.2e}" for e in per) + f"; momentum vector {mom:.2e})")
    # the bar: relative L1 of the whole conserved state and of every conserved
    # variable on its own norm
    assert err <= tol
    assert max(per) <= tol and mom <= tol
    g.close()


def _crossing(x, f, level):
    for i in range(len(f) - 1):
        if (f[i] - level) * (f[i + 1] - level) <= 0 and f[i] != f[i + 1]:
            return x[i] + (level - f[i]) / (f[i + 1] - f[i]) * (x[i + 1] - x[i])
    return None


def test_sod_fp32_shock_positions():
    need_gpu()
    n = 128
    pr = P.sod(n)
    o = oracle_sim(pr)
    o.advance(pr.t_end)
    announce("sod_fp32", pr.shape)
    g = gpu_sim(pr, "f32")
    g.advance(pr.t_end)
    ro = o.conserved()[0][0, 0]
    rg = g.conserved()[0][0, 0]
    x = (np.arange(n) + 0.5) / n
    for lev, lo, hi in [(0.9, 0.0, 0.5), (0.5, 0.3, 0.6), (0.346, 0.55, 0.8), (0.195, 0.75, 1.0)]:
        m = (x > lo) & (x < hi)
        assert abs(_crossing(x[m], rg[m], lev) - _crossing(x[m], ro[m], lev)) <= 1.0 / n
    assert rel_l1(rg, ro) <= 1e-4
    g.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_well_balanced_rest_gpu(dtype, tol):
    need_gpu()
    pr = P.well_rest(32, gamma=2.0)
    announce("wb_rest", dtype)
    g = gpu_sim(pr, dtype)
    g.advance(math.inf, 500)
    W = g.primitive()
    print(f"{dtype}: |u|max after 500 steps = {np.max(np.abs(W[1:4])):.3e}")
    assert np.max(np.abs(W[1:4])) <= tol
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_uniform_flow_bitwise(dtype):
    need_gpu()
    pr = P.uniform_flow((16, 12, 8))
    announce("uniform", dtype)
    g = gpu_sim(pr, dtype)
    U0 = g.conserved()
    g.advance(math.inf, 20)
    assert np.array_equal(g.conserved(), U0)
    g.close()


def test_conservation_periodic_gpu():
    need_gpu()
    pr = P.random_state((24, 20, 16), seed=3)
    announce("conservation")
    for dtype, tol in (("f64", 1e-13), ("f32", 2e-6)):
        g = gpu_sim(pr, dtype)
        g.step()
        T0 = g.totals()
        g.advance(math.inf, 50)
        T1 = g.totals()
        assert abs(T1[0] - T0[0]) <= tol * abs(T0[0])
        assert abs(T1[4] - T0[4]) <= tol * abs(T0[4])
        g.close()


def test_checkpoint_resume_and_determinism():
    need_gpu()
    pr = P.well_flow(20)
    announce("checkpoint")
    a = gpu_sim(pr, "f64")
    a.advance(math.inf, 20)
    b = gpu_sim(pr, "f64")
    b.advance(math.inf, 10)
    c = gpu_sim(pr, "f64")
    c.set_conserved(b.conserved())
    c.set_time(*b.time())
    c.advance(math.inf, 10)
    assert np.array_equal(a.conserved(), c.conserved())
    assert a.time() == c.time()
    d = gpu_sim(pr, "f64")
    d.advance(math.inf, 20)
    assert np.array_equal(a.conserved(), d.conserved())
    for s in (a, b, c, d):
        s.close()


def test_error_paths_sticky():
    need_gpu()
    from paper_1912_04855_amd._lib import CsphError, ERR_NONFINITE, ERR_STATE
    pr = P.uniform_flow((8, 8, 8))
    announce("errors")
    g = gpu_sim(pr, "f64")
    U = g.conserved()
    U[4, 3, 3, 3] = np.nan
    g.set_conserved(U)
    with pytest.raises(CsphError) as e:
        g.step()
    assert e.value.code == ERR_NONFINITE
    with pytest.raises(CsphError) as e:
        g.step()
    assert e.value.code == ERR_STATE
    g.set_primitive(pr.prim)
    g.step()
    g.close()


def test_torch_memory_and_stream():
    need_gpu()
    import torch
    pr = P.sod(64)
    o = oracle_sim(pr)
    o.advance(pr.t_end)
    announce("torch")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = gpu_sim(pr, "f64", torch=True)
        g.advance(pr.t_end)
        U = g.conserved()
    assert rel_l1_vars(U, o.conserved()) <= 1e-12
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_potential_cleared_equals_never_set(dtype):
    """Without a potential the kernels leave psi(r*) at 0 instead of interpolating
    it: a simulation whose potential is cleared after a few steps must then
    behave exactly like one that never had one."""
    need_gpu()
    pr = P.random_state((12, 10, 9), seed=7, potential=True,
                        bc=(P.OUTFLOW, P.OUTFLOW, P.REFLECT, P.REFLECT, P.PERIODIC, P.PERIODIC))
    flat = P.random_state((12, 10, 9), seed=7, potential=False,
                          bc=(P.OUTFLOW, P.OUTFLOW, P.REFLECT, P.REFLECT, P.PERIODIC, P.PERIODIC))
    announce("potential_cleared", dtype)
    a = gpu_sim(pr, dtype)
    a.advance(math.inf, 5)          # psi(r*) now holds nonzero values
    a.set_potential(None)
    a.set_primitive(flat.prim)
    a.set_time(0.0, 0)
    b = gpu_sim(flat, dtype)
    assert a.advance(math.inf, 20) == 20
    assert b.advance(math.inf, 20) == 20
    assert np.array_equal(a.conserved(), b.conserved())
    assert a.time() == b.time()
    if dtype == "f64":
        o = oracle_sim(flat)
        for _ in range(20):
            o.step()
        assert rel_l1_vars(a.conserved(), o.conserved()) <= 1e-12
    a.close()
    b.close()
