"""One GPU's z-slab share of a decomposed grid, on the GPU.

A slab carrying three overlap planes on either side (z faces OUTFLOW) advances
its owned planes exactly as the whole grid does, given the same dt: one step
reads U^n at most three cells away along an axis (the same property is pinned on
the oracle).  On the GPU the owned planes match the whole grid bit for bit in
FP64 and FP32, so the stage kernels compute a cell the same way whatever the
grid's extent in z and the sweep's place in it; checked on the headline
potential-well flow at 64^3 over two steps (the overlap refreshed between them,
as an exchange would) and at the real share of 256^3 over 8 GPUs, 256x256x38."""
import numpy as np
import pytest

from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu

pytestmark = pytest.mark.gpu


def _check(n, planes, k0, dtype, steps, dt):
    pr = P.well_flow(n)
    whole = gpu_sim(pr, dtype)
    whole.advance(np.inf, 3)  # a developed flow, not the uniform start
    H = 3
    ks = np.arange(k0, k0 + planes) % n
    ring = np.arange(k0 - H, k0 + planes + H) % n
    sl = P.z_slab(pr, k0, planes, H)
    part = gpu_sim(sl, dtype)
    part.set_conserved(P.z_cut(whole.conserved(), k0, planes, H))
    part.set_time(*whole.time())
    for s in range(steps):
        assert whole.step(dt_max=dt) == dt and part.step(dt_max=dt) == dt
        U, S = whole.conserved(), part.conserved()
        assert np.array_equal(S[:, H:H + planes], U[:, ks]), (s, dtype)
        S[:, :H] = U[:, ring[:H]]
        S[:, H + planes:] = U[:, ring[H + planes:]]
        part.set_conserved(S)
    whole.close()
    part.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k0", [0, 27])
def test_slab_share_matches_the_whole_grid(dtype, k0):
    need_gpu()
    announce("slab_share", dtype, k0)
    _check(64, 16, k0, dtype, 2, 2e-4)


def test_real_share_of_256():
    need_gpu()
    announce("slab_share_256")
    _check(256, 32, 96, "f32", 1, 5e-5)
