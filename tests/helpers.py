"""Shared test helpers: build an oracle sim from a problem description."""
import math

import numpy as np

import oracle as O


def oracle_sim(prob, **kw):
    s = O.OracleSim(prob.shape, prob.h, gamma=prob.gamma, cfl=prob.cfl, rho_vac=prob.rho_vac,
                    bc=prob.bc, inflow=prob.inflow_list(), origin=prob.origin,
                    **dict({"nu": prob.nu, "grav": prob.grav}, **kw))
    s.set_primitive(prob.prim)
    s.set_potential(prob.psi)
    if prob.src is not None:
        s.set_source(prob.src, prob.eps_src)
    return s


def l1_rel(a, b):
    """Relative L1 distance sum|a-b| / sum|b| over all components."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sum(np.abs(b))
    return float(np.sum(np.abs(a - b)) / den) if den > 0 else float(np.sum(np.abs(a - b)))


def l1_rel_per_var(a, b):
    return [l1_rel(a[v], b[v]) for v in range(a.shape[0])]


def orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def golden(name):
    """Values of a fixture under tests/golden/ (``key value`` lines, '#' comments)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    out = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            out[k] = float(v)
    return out
