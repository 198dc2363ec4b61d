"""Boundary rules on the x faces at awkward sizes.  The FP32 build writes the
x-face ghost cells from the stage that produces each field (the FP64 build fills
them in the fill kernels), so every x rule -- periodic wrap, reflect mirror,
outflow copy, inflow state -- is checked in both precisions: on grids 4 and 5
cells wide (every cell is then a ghost source, for both faces at once) and on a
grid whose width leaves a ragged last tile, against the FP64 oracle (FP64 to
1e-12 relative L1 per variable; FP32 to 1e-5 on a smooth state)."""
import math

import pytest

from paper_1912_04855_amd import problems as P

from gpu_common import announce, gpu_sim, need_gpu, rel_l1_vars
from helpers import oracle_sim

pytestmark = pytest.mark.gpu

X_RULES = {
    "periodic": (P.PERIODIC, P.PERIODIC),
    "reflect": (P.REFLECT, P.REFLECT),
    "outflow_inflow": (P.OUTFLOW, P.INFLOW),
    "inflow_reflect": (P.INFLOW, P.REFLECT),
    "reflect_outflow": (P.REFLECT, P.OUTFLOW),
}
SHAPES = [(4, 6, 5), (5, 9, 7), (37, 10, 9)]


def _problem(rule, shape, seed):
    bc = X_RULES[rule] + (P.PERIODIC, P.PERIODIC, P.REFLECT, P.OUTFLOW)
    pr = P.smooth_state(shape, seed=seed, bc=bc)
    pr.inflow = {0: (1.05, 0.25, 0.02, -0.03, 1.1), 1: (0.95, -0.2, 0.01, 0.02, 0.9)}
    return pr


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("rule", list(X_RULES))
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_x_face_rules(rule, shape, dtype, tol):
    need_gpu()
    pr = _problem(rule, shape, seed=len(rule) + shape[0])
    steps = 15
    o = oracle_sim(pr)
    for _ in range(steps):
        o.step()
    announce("x_face_rules", rule, shape, dtype)
    g = gpu_sim(pr, dtype)
    assert g.advance(math.inf, steps) == steps
    err = rel_l1_vars(g.conserved(), o.conserved())
    assert err <= tol, err
    g.close()
