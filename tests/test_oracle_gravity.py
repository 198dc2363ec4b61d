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
  * a uniform gas feels no self-gravity; partly periodic boxes are refused;
  * isolated boxes (no periodic face): the self term of a cell is the integral
    of 1/|x| over its cube (against numerical quadrature), the potential at the
    centre of a uniform cube converges to the continuum value at second order,
    the far field is the monopole, and a cold uniform sphere falls in at the
    Newtonian rate -(4/3) pi G rho r.
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


@pytest.mark.parametrize("axis", range(3))
def test_self_gravity_refuses_a_partly_periodic_box(axis):
    bc = [P.PERIODIC] * 6
    bc[2 * axis] = bc[2 * axis + 1] = P.REFLECT
    with pytest.raises(RuntimeError):
        O.OracleSim((8, 8, 8), 0.1, bc=tuple(bc), grav=1.0)
    with pytest.raises(RuntimeError):
        O.OracleSim((8, 8, 8), 0.1, grav=-1.0)


# --------------------------------------------------------------- isolated boxes
# Reading: with no periodic face the gas's potential is that of its mass in free
# space, psi_i = -G h^3 sum_j rho_j phi_ij with phi = 1/|r_i - r_j| between
# cells and C/h within a cell, C the integral of 1/|x| over a unit cube.

def _isolated(n, G=1.0):
    return O.OracleSim((n, n, n), 1.0 / n, bc=(P.OUTFLOW,) * 6, grav=G)


def test_isolated_self_term_is_the_cube_integral():
    from scipy import integrate
    quad, _ = integrate.tplquad(lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z),
                                0, 0.5, 0, 0.5, 0, 0.5, epsabs=1e-12, epsrel=1e-12)
    n, G = 8, 0.7
    o = _isolated(n, G)
    rho = np.zeros((n, n, n))
    rho[3, 4, 5] = 2.0
    psi = o.self_potential(rho)
    h = 1.0 / n
    assert psi[3, 4, 5] == pytest.approx(-G * 2.0 * h * h * 8 * quad, rel=1e-9)


def test_isolated_cube_centre_potential_converges_at_second_order():
    # the potential at the centre of a uniform unit cube is -G rho C (C = the
    # integral of 1/|x| over it); the sum over n^3 cells converges to it
    C = 3 * math.log(2 + math.sqrt(3)) - math.pi / 2
    errs = []
    for n in (4, 8, 16):
        psi = _isolated(n).self_potential(np.ones((n, n, n)))
        c = n // 2
        errs.append(abs(psi[c - 1:c + 1, c - 1:c + 1, c - 1:c + 1].mean() + C))
    assert min(orders(errs)) >= 1.9
    assert errs[-1] <= 0.01 * C


def test_isolated_far_field_is_the_monopole():
    n, G = 16, 1.3
    o = _isolated(n, G)
    rho = np.zeros((n, n, n))
    rho[:3, :3, :3] = 1.5
    psi = o.self_potential(rho)
    h = 1.0 / n
    M = 1.5 * 27 * h ** 3
    centre = np.array([1.5, 1.5, 1.5]) * h
    far = (np.array([n - 1, n - 1, n - 1]) + 0.5) * h
    expect = -G * M / np.linalg.norm(far - centre)
    # the quadrupole of a cube vanishes: the first correction is (L / r)^4
    assert psi[n - 1, n - 1, n - 1] == pytest.approx(expect, rel=2e-4)


def test_cold_sphere_falls_in_at_the_newtonian_rate():
    # a cold uniform sphere in vacuum: at first every shell falls with
    # acceleration -G M(r) / r^2 = -(4/3) pi G rho r
    n, G = 16, 1.0
    pr = P.cold_sphere(n, R=0.3, G=G)
    x, y, z = P.centres(pr.shape, pr.h)
    r = np.broadcast_to(np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), (n, n, n))
    o = oracle_sim(pr)
    for _ in range(3):
        o.step(dt_max=0.01)
    t = o.time()[0]
    U = o.conserved()
    off = [np.broadcast_to(c - 0.5, (n, n, n)) for c in (x, y, z)]
    ur = (U[1] * off[0] + U[2] * off[1] + U[3] * off[2]) / r / U[0]
    sel = (r > 0.08) & (r < 0.2)
    ratio = ur[sel] / (-(4 / 3) * math.pi * G * r[sel] * t)
    assert abs(ratio.mean() - 1.0) <= 0.01
    assert np.all(np.abs(ratio - 1.0) <= 0.03)


def test_potential_at_sampled_cells():
    n = 10
    o = O.OracleSim((n, 8, 6), 0.1, bc=(P.OUTFLOW,) * 6, grav=0.8)
    rho = np.random.default_rng(4).uniform(0.1, 2.0, (6, 8, n))
    full = o.self_potential(rho)
    cells = [(0, 0, 0), (9, 7, 5), (3, 4, 2)]
    got = o.self_potential_at(rho, cells)
    assert np.array_equal(got, [full[k, j, i] for i, j, k in cells])
    with pytest.raises(O.OracleError):
        o.self_potential_at(rho, [(10, 0, 0)])


def test_self_gravity_box_classes():
    # all faces periodic (spectral solve) or none (free space); a mix is refused
    O.OracleSim((8, 8, 8), 0.1, bc=(P.OUTFLOW, P.INFLOW, P.REFLECT, P.REFLECT, P.OUTFLOW, P.OUTFLOW),
                grav=1.0)
    with pytest.raises(RuntimeError):
        O.OracleSim((8, 8, 8), 0.1, bc=(P.OUTFLOW, P.OUTFLOW) + (P.PERIODIC,) * 4, grav=1.0)
