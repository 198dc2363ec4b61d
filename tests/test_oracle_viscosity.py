"""Pins of the viscous extension (Sec. 4: viscous flows) of the oracle.

A shear wave u_y = A sin(2 pi x) in a uniform gas at rest otherwise is a
solution of the viscous equations in which the pressure stays uniform and the
amplitude decays as exp(-nu k^2 t), k = 2 pi (the diffusion of momentum).  The
scheme's lattice Laplacian acts on it as the three-point one, so the measured
decay rate must converge to nu k^2 at second order.  The viscous force and its
work are pairwise antisymmetric: momentum and total energy stay exact on a
periodic box while kinetic energy turns into heat."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1912_04855_amd import problems as P

from helpers import orders


def _shear(n, nu, A=1e-3, t_end=0.5):
    shape = (n, 4, 4)
    h = 1.0 / n
    x, _, _ = P.centres(shape, h)
    prim = np.zeros((5, 4, 4, n))
    prim[0] = 1.0
    prim[4] = 1.0
    prim[2] = np.broadcast_to(A * np.sin(2 * math.pi * x), prim.shape[1:])
    s = O.OracleSim(shape, h, gamma=1.4, cfl=0.4, bc=(P.PERIODIC,) * 6, nu=nu)
    s.set_primitive(prim)
    s.advance(t_end)
    xc = (np.arange(n) + 0.5) / n
    amp = 2 * np.mean(s.primitive()[2][0, 0, :] * np.sin(2 * math.pi * xc))
    amp0 = 2 * np.mean(prim[2][0, 0, :] * np.sin(2 * math.pi * xc))
    return -math.log(amp / amp0) / t_end


@pytest.mark.slow
def test_shear_wave_decays_at_the_viscous_rate():
    nu = 0.01
    exact = nu * (2 * math.pi) ** 2
    rates = [_shear(n, nu) for n in (32, 64, 128)]
    err = [abs(r - exact) / exact for r in rates]
    # measured 6.5e-2, 1.4e-2, 3.4e-3: second order
    assert err[-1] < 5e-3, rates
    assert min(orders(err)) >= 1.8, err
    # without viscosity the same wave hardly decays (the face flux's damping of
    # the velocity jump of the reconstructed states only): 0.0015 at 128 cells
    assert _shear(128, 0.0) < 0.01 * exact


def test_viscous_conservation_and_heating():
    pr = P.random_state((12, 10, 8), seed=21)
    s = O.OracleSim(pr.shape, pr.h, gamma=pr.gamma, cfl=pr.cfl, bc=(P.PERIODIC,) * 6, nu=0.02)
    s.set_primitive(pr.prim)
    t = O.OracleSim(pr.shape, pr.h, gamma=pr.gamma, cfl=pr.cfl, bc=(P.PERIODIC,) * 6, nu=0.0)
    t.set_primitive(pr.prim)
    h3 = pr.h ** 3
    U0 = s.conserved()
    ke0 = 0.5 * np.sum((U0[1] ** 2 + U0[2] ** 2 + U0[3] ** 2) / U0[0]) * h3
    for _ in range(20):
        dt = s.step()
        t.step(dt_max=dt)
    U1, V1 = s.conserved(), t.conserved()
    tot0 = np.sum(U0, axis=(1, 2, 3)) * h3
    tot1 = np.sum(U1, axis=(1, 2, 3)) * h3
    scale = np.array([tot0[0], 1.0, 1.0, 1.0, tot0[4]])
    np.testing.assert_allclose(tot1, tot0, rtol=0, atol=1e-13 * np.max(np.abs(scale)))
    # the viscous run has less kinetic energy than the inviscid one at the same times
    ke_v = 0.5 * np.sum((U1[1] ** 2 + U1[2] ** 2 + U1[3] ** 2) / U1[0]) * h3
    ke_i = 0.5 * np.sum((V1[1] ** 2 + V1[2] ** 2 + V1[3] ** 2) / V1[0]) * h3
    assert ke_v < ke_i < ke0


def test_viscous_time_step_limit():
    # nu dt <= h^2 / 4: with a large viscosity the step is the viscous one
    pr = P.uniform_flow((8, 8, 8), u=(0.1, 0.0, 0.0))
    nu = 10.0
    s = O.OracleSim(pr.shape, pr.h, gamma=pr.gamma, cfl=pr.cfl, bc=(P.PERIODIC,) * 6, nu=nu)
    s.set_primitive(pr.prim)
    assert s.step() == pytest.approx(0.25 * pr.h ** 2 / nu, rel=1e-15)
    with pytest.raises(O.OracleError):
        O.OracleSim(pr.shape, pr.h, bc=(P.PERIODIC,) * 6, nu=-1.0)


def test_viscous_force_and_work_rates_match_the_continuum():
    """Over a vanishing step of the shear wave u_y = A sin(k x) (uniform density and
    pressure, no other motion) the momentum changes at the viscous force
    rho nu u_y'' = -rho nu k^2 A sin(k x) and the energy at the work of the
    viscous stress, div(rho nu grad(|u|^2/2)) = rho nu A^2 k^2 cos(2 k x); the
    inviscid parts of Q cancel exactly here (u varies along x only).  Both rates
    converge to these at second order (the lattice Laplacian is the three-point
    one for such fields).  The same step without viscosity is subtracted: it
    carries the face flux's damping of the velocity jumps of the reconstructed
    states, which is independent of nu."""
    n, A, nu, dt = 64, 0.1, 0.01, 1e-7
    k = 2 * math.pi
    shape = (n, 4, 4)
    h = 1.0 / n
    x, _, _ = P.centres(shape, h)
    prim = np.zeros((5, 4, 4, n))
    prim[0] = 1.0
    prim[4] = 1.0
    prim[2] = np.broadcast_to(A * np.sin(k * x), prim.shape[1:])
    U = []
    for v in (nu, 0.0):
        s = O.OracleSim(shape, h, gamma=1.4, cfl=0.4, bc=(P.PERIODIC,) * 6, nu=v)
        s.set_primitive(prim)
        assert s.step(dt_max=dt) == dt
        U.append(s.conserved())
    xc = (np.arange(n) + 0.5) / n
    force = (U[0][2] - U[1][2])[0, 0] / dt
    work = (U[0][4] - U[1][4])[0, 0] / dt
    f_ex = -nu * k * k * A * np.sin(k * xc)
    w_ex = nu * A * A * k * k * np.cos(2 * k * xc)
    # the three-point Laplacian of sin(k x) and cos(2 k x): relative errors
    # (k h)^2/12 = 8e-4 and (2 k h)^2/12 = 3.2e-3
    assert np.max(np.abs(force - f_ex)) <= 2e-3 * np.max(np.abs(f_ex))
    assert np.max(np.abs(work - w_ex)) <= 6e-3 * np.max(np.abs(w_ex))
