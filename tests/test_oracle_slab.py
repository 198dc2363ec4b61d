"""The z-slab share that one GPU of a decomposed grid would hold.

One step of the method reads U^n at most three cells away along an axis: stage
E's face reconstruction reaches two cells of U^n and one of the corrector's
results, which read the predictor's one cell further out, which read U^n one
cell further again.  So a slab that carries three overlap planes on either side
(its own z faces given any rule) advances its owned planes exactly as the whole
grid does, given the same dt; the overlap planes are then stale and would be
refreshed from the neighbouring slabs.  Checked on the oracle: bit for bit with
three overlap planes over two steps (the overlap refreshed between them), and
not with two."""
import numpy as np
import pytest

from paper_1912_04855_amd import problems as P

from helpers import oracle_sim


def _whole():
    pr = P.random_state((12, 10, 16), seed=6, potential=True)
    o = oracle_sim(pr)
    for _ in range(2):
        o.step()
    return pr, o


@pytest.mark.parametrize("k0", [0, 5, 12])
def test_slab_with_three_overlap_planes_is_exact(k0):
    pr, whole = _whole()
    L, H = 6, 3
    nz = pr.shape[2]
    ks = np.arange(k0, k0 + L) % nz
    ring = np.arange(k0 - H, k0 + L + H) % nz
    sl = P.z_slab(pr, k0, L, H)
    o = oracle_sim(sl)
    o.set_conserved(P.z_cut(whole.conserved(), k0, L, H))
    for step in range(2):
        dt = 0.5 * min(whole.cfl_dt(), o.cfl_dt())
        assert whole.step(dt_max=dt) == dt and o.step(dt_max=dt) == dt
        U, S = whole.conserved(), o.conserved()
        assert np.array_equal(S[:, H:H + L], U[:, ks]), step
        # the exchange: the overlap planes from the neighbours, the owned ones kept
        S[:, :H] = U[:, ring[:H]]
        S[:, H + L:] = U[:, ring[H + L:]]
        o.set_conserved(S)


def test_two_overlap_planes_are_not_enough():
    pr, whole = _whole()
    L, H = 6, 2
    U = whole.conserved()
    sl = P.z_slab(pr, 4, L, H)
    o = oracle_sim(sl)
    o.set_conserved(P.z_cut(U, 4, L, H))
    dt = 0.5 * min(whole.cfl_dt(), o.cfl_dt())
    whole.step(dt_max=dt)
    o.step(dt_max=dt)
    ks = np.arange(4, 4 + L)
    got, want = o.conserved()[:, H:H + L], whole.conserved()[:, ks]
    assert not np.array_equal(got[:, 0], want[:, 0]) and not np.array_equal(got[:, -1], want[:, -1])
    assert np.array_equal(got[:, 2:-2], want[:, 2:-2])
