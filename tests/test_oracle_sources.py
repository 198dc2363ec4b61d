"""Pins of the sources-and-sinks extension (Sec. 4: non-stationary sources and
sinks) of the oracle.

Reading: a mass rate q per cell, which the caller may change between steps; a
source (q > 0) injects gas at rest with specific internal energy eps, a sink
(q < 0) removes gas at the local specific values (limited at zero); the step
applies half of it before and half after the hydrodynamic step.  The pins:
  * closed forms where the hydrodynamics does nothing (uniform states): a source
    in gas at rest and in uniform flow (rho = rho0 + q t, momentum unchanged,
    E = E0 + q eps t), a sink (rho = rho0 + q t with u and E/rho unchanged), and
    a sink that empties the box (exact zeros, never negative);
  * the mass budget of a random source field on a periodic box (total mass
    grows by sum(q) h^3 t; momentum is untouched by injection at rest);
  * the splitting: one step equals half the source, a source-free step of the
    same dt, and half the source again (a scheme that applies the whole source
    after the step fails this);
  * a change of q between steps takes effect from the next step;
  * convergence under joint refinement on a smooth source and sink pair.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1912_04855_amd import problems as P

from helpers import oracle_sim, orders


def _uniform(u=(0.0, 0.0, 0.0), shape=(8, 8, 8)):
    return P.uniform_flow(shape, u=u, rho=1.0, p=1.0, gamma=1.4)


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.1)])
def test_source_in_uniform_gas(u):
    q, eps = 0.5, 2.0
    o = oracle_sim(_uniform(u))
    o.set_source(q, eps)
    U0 = o.conserved()
    o.advance(0.3)
    t = o.time()[0]
    U = o.conserved()
    assert np.max(np.abs(U[0] - (1.0 + q * t))) <= 1e-14
    assert np.max(np.abs(U[1:4] - U0[1:4])) <= 1e-15
    assert np.max(np.abs(U[4] - (U0[4] + q * eps * t))) <= 1e-14


def test_sink_keeps_velocity_and_specific_energy():
    q = -0.5
    o = oracle_sim(_uniform((0.3, -0.2, 0.1)))
    o.set_source(q, 0.0)
    U0 = o.conserved()
    o.advance(0.6)
    t = o.time()[0]
    U = o.conserved()
    assert np.max(np.abs(U[0] - (1.0 + q * t))) <= 1e-14
    assert np.max(np.abs(U[1:4] / U[0] - U0[1:4] / U0[0])) <= 1e-14
    assert np.max(np.abs(U[4] / U[0] - U0[4] / U0[0])) <= 1e-14


def test_sink_empties_to_exact_zero():
    o = oracle_sim(_uniform((0.3, -0.2, 0.1)))
    o.set_source(-5.0, 0.0)
    for _ in range(10):
        o.step(dt_max=0.05)  # the box runs out of gas: no signal speed is left
    U = o.conserved()
    assert np.all(U == 0.0)


def test_mass_budget_of_a_random_source_field():
    pr = P.random_state((12, 10, 8), seed=5)
    o = oracle_sim(pr)
    q = np.random.default_rng(3).uniform(0.0, 2.0, o.shape)
    o.set_source(q, 1.0)
    U0 = o.conserved()
    o.advance(0.05)
    t = o.time()[0]
    U = o.conserved()
    assert abs(U[0].sum() - (U0[0].sum() + q.sum() * t)) <= 1e-12 * U0[0].sum()
    for d in (1, 2, 3):
        assert abs(U[d].sum() - U0[d].sum()) <= 1e-12 * np.abs(U0[d]).sum()


def _half_source(U, q, eps, hdt):
    """Half a step of the source, cell by cell, as the reading states it."""
    U = U.copy()
    d = hdt * q
    src = q > 0
    U[0][src] += d[src]
    U[4][src] += d[src] * eps
    snk = (q < 0) & (U[0] > 0)
    rn = np.maximum(U[0][snk] + d[snk], 0.0)
    f = rn / U[0][snk]
    for v in (1, 2, 3, 4):
        U[v][snk] *= f
    U[0][snk] = rn
    return U


def test_step_is_half_source_hydro_half_source():
    pr = P.smooth_state((10, 8, 6), seed=2, potential=True)
    dt = 2e-3  # below the CFL step, so both runs take it
    q = np.where(np.arange(480).reshape(6, 8, 10) % 3 == 0, -0.7, 1.3)
    eps = 0.8
    a = oracle_sim(pr)
    a.set_source(q, eps)
    assert a.step(dt_max=dt) == dt
    b = oracle_sim(pr)
    b.set_conserved(_half_source(b.conserved(), q, eps, 0.5 * dt))
    assert b.step(dt_max=dt) == dt
    Ub = _half_source(b.conserved(), q, eps, 0.5 * dt)
    assert np.max(np.abs(a.conserved() - Ub)) <= 1e-13 * np.max(np.abs(Ub))


def test_changing_the_source_between_steps():
    o = oracle_sim(_uniform())
    o.set_source(1.0, 1.0)
    t1 = o.step(dt_max=0.01)
    o.set_source(-0.5, 0.0)
    t2 = o.step(dt_max=0.01)
    o.set_source(None)
    o.step(dt_max=0.01)
    rho = o.conserved()[0]
    assert np.max(np.abs(rho - (1.0 + t1) * (1.0 - 0.5 * t2 / (1.0 + t1)))) <= 1e-14


def _source_pair(n):
    shape = (n, 4, 4)
    h = 1.0 / n
    x, _, _ = P.centres(shape, h)
    prim = np.zeros((5, 4, 4, n))
    prim[0] = 1.0
    prim[4] = 1.0
    pr = P.Problem("source_pair", shape, h, 1.4, 0.4, (P.PERIODIC,) * 6, prim)
    o = oracle_sim(pr)
    q = 2.0 * np.exp(-(x - 0.5) ** 2 / 0.01) - np.exp(-(x - 0.2) ** 2 / 0.005)
    o.set_source(np.broadcast_to(q, (4, 4, n)), 1.5)
    o.advance(0.2)
    return o.conserved()[:, 0, 0, :]


def test_source_pair_converges():
    ref = _source_pair(512)
    errs = []
    for n in (64, 128, 256):
        f = 512 // n
        r = ref.reshape(5, n, f).mean(axis=2)
        errs.append(float(np.abs(_source_pair(n) - r).sum() / np.abs(r).sum()))
    print("source pair: errors", errs, "orders", orders(errs))
    assert min(orders(errs)) >= 1.8


def test_bad_sources_are_refused():
    o = oracle_sim(_uniform())
    with pytest.raises(O.OracleError):
        o.set_source(np.full(o.shape, np.nan), 1.0)
    with pytest.raises(O.OracleError):
        o.set_source(1.0, -1.0)
