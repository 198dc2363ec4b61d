"""Pins of the self-gravity extension (Sec. 4: the gas's self-gravity) of the
oracle.

Reading: on a periodic box the gas's potential solves the 7-point discrete
Poisson equation L7[psi] = 4 pi G (rho - mean rho); the predictor takes the
potential of rho^n, the corrector that of the density the continuity equation
predicts for t^{n+1}.  The pins:
  * a single Fourier mode has the closed-form potential 4 pi G delta cos(k.x) /
    lambda(k), lambda the eigenvalue of L7 (checks each axis, the eigenvalue,
    the normalisation and the sign);
  * for a random density, L7 of the result, taken by finite differences, equals
    4 pi G (rho - mean rho) cell by cell and the potential has zero mean;
  * a linear Jeans wave follows the dispersion relation omega^2 = c^2 k^2 -
    4 pi G rho0 (oscillation below the Jeans scale, cosh growth above it) with
    second-order convergence under joint refinement of h and dt; a corrector
    that kept the potential of rho^n converges at first order here (measured
    1.1), so this pin separates the two readings;
  * the stage fields: the potential of the step is the external one plus the
    self potential of rho^n, and the corrector's is that of the predicted
    density;
  * a uniform gas feels no self-gravity; non-periodic faces are refused.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1912_04855_amd import problems as P

from helpers import oracle_sim, orders


def _grid(nx=16, ny=8, nz=4):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z


@pytest.mark.parametrize("mode", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (3, 2, 1), (8, 4, 2), (5, 7, 3)])
def test_single_mode_has_the_closed_form_potential(mode):
    nx, ny, nz = 16, 8, 4
    h, G, delta = 0.1, 0.7, 0.3
    o = O.OracleSim((nx, ny, nz), h, grav=G)
    x, y, z = _grid(nx, ny, nz)
    a, b, c = mode
    phase = 2 * math.pi * (a * x / nx + b * y / ny + c * z / nz)
    rho = 2.0 + delta * np.cos(phase)
    lam = sum((2 * math.cos(2 * math.pi * k / n) - 2) / h ** 2
              for k, n in ((a, nx), (b, ny), (c, nz)))
    exact = 4 * math.pi * G * delta * np.cos(phase) / lam
    got = o.self_potential(rho)
    assert np.max(np.abs(got - exact)) <= 1e-12 * np.max(np.abs(exact))
    # attraction: the potential is lowest where the density is highest
    assert got.flat[np.argmax(rho)] < 0.0


def test_potential_solves_the_discrete_poisson_equation():
    nx, ny, nz = 12, 10, 6
    h, G = 0.05, 1.3
    o = O.OracleSim((nx, ny, nz), h, grav=G)
    rho = np.random.default_rng(7).uniform(0.5, 2.0, (nz, ny, nx))
    psi = o.self_potential(rho)
    lap = sum((np.roll(psi, 1, ax) + np.roll(psi, -1, ax) - 2 * psi) / h ** 2 for ax in range(3))
    src = 4 * math.pi * G * (rho - rho.mean())
    assert np.max(np.abs(lap - src)) <= 1e-12 * np.max(np.abs(src))
    assert abs(psi.mean()) <= 1e-14 * np.max(np.abs(psi))


def _jeans_amplitude(n, G, axis=0, t_end=0.5, delta=1e-5):
    pr = P.jeans_wave(n, G, delta=delta, axis=axis, t_end=t_end)
    o = oracle_sim(pr)
    o.advance(pr.t_end)
    rho = o.conserved()[0]
    x = (np.arange(n) + 0.5) / n
    line = np.moveaxis(rho, 2 - axis, -1).reshape(-1, n)[0]
    return 2 * np.mean((line - 1.0) * np.cos(2 * math.pi * x)) / delta


def _jeans_exact(G, t):
    w2 = (2 * math.pi) ** 2 - 4 * math.pi * G   # c = 1, rho0 = 1, k = 2 pi
    return math.cos(math.sqrt(w2) * t) if w2 > 0 else math.cosh(math.sqrt(-w2) * t)


@pytest.mark.parametrize("G,axis", [(math.pi / 2, 0), (2 * math.pi, 0), (2 * math.pi, 1)])
def test_jeans_wave_follows_the_dispersion_relation_at_second_order(G, axis):
    # G = pi/2: 4 pi G rho0 = c^2 k^2 / 2, an oscillation; G = 2 pi: 4 pi G rho0 =
    # 2 c^2 k^2, growth at sigma = c k
    exact = _jeans_exact(G, 0.5)
    errs = [abs(_jeans_amplitude(n, G, axis) - exact) for n in (16, 32, 64)]
    print(f"Jeans G={G:.4f} axis {axis}: errors {errs}, orders {orders(errs)}")
    assert min(orders(errs)) >= 1.8
    assert errs[-1] <= 0.015 * abs(exact)


def test_stage_potentials():
    pr = P.random_state((12, 10, 8), seed=3, potential=True)
    pr.grav = 0.5
    o = oracle_sim(pr)
    U = o.conserved()
    dt = o.step()
    psi_self = o.self_potential(U[0])
    assert np.allclose(o.field("psi"), pr.psi + psi_self, rtol=0, atol=1e-13)
    # the corrector's potential: that of the density predicted for t^{n+1}
    h = pr.h
    div = sum((np.roll(U[1 + d], -1, 2 - d) - np.roll(U[1 + d], 1, 2 - d)) / (2 * h) for d in range(3))
    psi_hat = o.self_potential(U[0] - dt * div)
    assert np.allclose(o.field("psih"), pr.psi + psi_hat, rtol=0, atol=1e-13)
    assert np.max(np.abs(psi_hat - psi_self)) > 1e-3 * np.max(np.abs(psi_self))


def test_uniform_gas_stays_at_rest():
    pr = P.uniform_flow((8, 8, 8), u=(0.0, 0.0, 0.0))
    pr.grav = 1.0
    o = oracle_sim(pr)
    for _ in range(5):
        o.step()
    U = o.conserved()
    assert np.max(np.abs(U[1:4])) <= 1e-14
    assert np.max(np.abs(U[0] - 1.0)) <= 1e-14


@pytest.mark.parametrize("face", range(6))
def test_self_gravity_needs_a_periodic_box(face):
    bc = [P.PERIODIC] * 6
    bc[face] = P.REFLECT
    with pytest.raises(RuntimeError):
        O.OracleSim((8, 8, 8), 0.1, bc=tuple(bc), grav=1.0)
    with pytest.raises(RuntimeError):
        O.OracleSim((8, 8, 8), 0.1, grav=-1.0)
