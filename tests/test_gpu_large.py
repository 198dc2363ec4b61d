"""Large grids through the box entry points (csph_fill_state, csph_set_state_box,
csph_get_state_box): box writes and reads agree with the whole-state calls, and
a 1024^3 FP32 grid (4.3 GB per field: byte offsets beyond 32 bits) evolves a
pulse near its far corner to the same bits as a 64^3 grid does at its centre."""
import math
import time

import numpy as np
import pytest

from paper_1912_04855_amd import _lib
from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu

pytestmark = pytest.mark.gpu


def _sim(shape, dtype, h=None):
    from paper_1912_04855_amd.sim import Sim
    return Sim(shape, h or 1.0 / shape[0], gamma=1.4, dtype=dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_box_io_matches_whole_state(dtype):
    need_gpu()
    pr = P.random_state((20, 12, 10), seed=12, potential=True)
    announce("box_io", dtype)
    a = gpu_sim(pr, dtype)
    b = gpu_sim(pr, dtype)
    lo, n = (3, 2, 1), (9, 7, 5)
    U = a.conserved()
    box = a.get_box(lo, n)
    assert np.array_equal(box, U[:, 1:6, 2:9, 3:12])
    prim = a.get_box(lo, n, vars=_lib.PRIMITIVE)
    new = prim.copy()
    new[0] *= 1.3
    new[4] *= 0.7
    a.set_box(lo, new)
    # the same change through the whole-state call, in conserved variables formed
    # as the library forms them
    cons = np.empty_like(new)
    cons[0] = new[0]
    for d in range(3):
        cons[1 + d] = new[0] * new[1 + d]
    cons[4] = new[4] / (pr.gamma - 1.0) + 0.5 * new[0] * (
        new[1] * new[1] + new[2] * new[2] + new[3] * new[3])
    Ub = U.copy()
    Ub[:, 1:6, 2:9, 3:12] = cons
    b.set_state(Ub, vars=_lib.CONSERVED)
    assert np.array_equal(a.conserved(), b.conserved())
    for s in (a, b):
        assert s.advance(math.inf, 5) == 5
    assert np.array_equal(a.conserved(), b.conserved())
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fill_state_matches_set_state(dtype):
    need_gpu()
    announce("fill_state", dtype)
    st = np.array([1.2, 0.3, -0.2, 0.1, 0.9])
    a = _sim((16, 8, 8), dtype)
    a.fill_state(st)
    b = _sim((16, 8, 8), dtype)
    b.set_state(np.broadcast_to(st[:, None, None, None], (5, 8, 8, 16)).copy())
    assert np.array_equal(a.conserved(), b.conserved())
    for s in (a, b):
        s.set_time(0.0, 0)
        assert s.advance(math.inf, 4) == 4
    assert np.array_equal(a.conserved(), b.conserved())
    a.close()
    b.close()


def test_box_refusals():
    need_gpu()
    announce("box_refusals")
    a = _sim((16, 8, 8), "f32")
    a.fill_state(np.array([1.0, 0.0, 0.0, 0.0, 1.0]))
    with pytest.raises(_lib.CsphError):
        a.get_box((10, 0, 0), (7, 1, 1))
    with pytest.raises(_lib.CsphError):
        a.set_box((0, 0, -1), np.ones((5, 1, 1, 1)))
    with pytest.raises(_lib.CsphError):
        a.fill_state(np.array([-1.0, 0.0, 0.0, 0.0, 1.0]))
    a.close()


def _pulse(n=16):
    """rho and p raised by a smooth bump over an n^3 box (primitive, [5, n, n, n])."""
    x = (np.arange(n) + 0.5) / n - 0.5
    r2 = x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2
    bump = np.exp(-r2 / 0.02)
    w = np.empty((5, n, n, n))
    w[0] = 1.0 + 0.5 * bump
    w[1], w[2], w[3] = 0.3, -0.2, 0.1
    w[4] = 1.0 + 0.8 * bump
    return w


def test_max_size_pulse_matches_small_grid():
    need_gpu()
    background = np.array([1.0, 0.3, -0.2, 0.1, 1.0])
    out = {}
    for N, lo in ((64, 24), (1024, 992)):
        announce("max_size_pulse", N)
        s = _sim((N, N, N), "f32", h=1.0 / 64)  # one cell size for both grids
        s.fill_state(background)
        s.set_box((lo, lo, lo), _pulse())
        t0 = time.time()
        assert s.advance(math.inf, 2) == 2
        dt = s.time()[0]
        wall = time.time() - t0
        out[N] = (s.get_box((lo - 12, lo - 12, lo - 12), (40, 40, 40)), dt)
        print(f"{N}^3 FP32: 2 steps to t = {dt:.6e} in {wall:.2f} s", flush=True)
        s.close()
    assert out[64][1] == out[1024][1]
    assert np.array_equal(out[64][0], out[1024][0])
    # the pulse did move the gas
    assert np.max(np.abs(out[64][0][1] - 0.3)) > 1e-3
