"""Pins of the oracle's building blocks against mathematics that fixes them.

Smoothing kernel (Eq. (7), kernel form left open in Sec. 4): the gradient must be
the derivative of the textbook M4 spline, odd, radial and compactly supported, and
its normalisation must make the 27-point sum exact for every polynomial of degree
<= 2.  Limiters (Sec. 2.2, TVD condition), the equation of state (Sec. 2.1), the
ghost-cell rules and the trilinear potential are pinned by their definitions.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1912_04855_amd import problems as P

from helpers import oracle_sim


# ---------------------------------------------------------------- kernel
def m4(q):
    """Textbook M4 cubic spline shape (un-normalised), support 2."""
    q = abs(q)
    if q < 1:
        return 1 - 1.5 * q * q + 0.75 * q ** 3
    if q < 2:
        return 0.25 * (2 - q) ** 3
    return 0.0


@pytest.mark.parametrize("d", [(-1, 0, 0), (0.3, -0.2, 0.1), (0.9, 0.9, 0.2), (1.2, -0.7, 0.4),
                               (0.05, 0.0, 0.0), (1.0, 1.0, 1.0)])
def test_kernel_gradient_is_m4_derivative(d):
    h = 0.37
    d = np.array(d, float) * h
    r = np.linalg.norm(d)
    q = r / h
    e = 1e-6
    dfdq = (m4(q + e) - m4(q - e)) / (2 * e)
    K = O.kernel_grad(d, h)
    kappa = O.kappa()
    # grad_i W(r_i - r_j) = (kappa/h) f'(q) d/|d|
    np.testing.assert_allclose(K, kappa / h * dfdq * d / r, rtol=1e-8, atol=1e-12)


def test_kernel_odd_radial_support():
    h = 0.5
    rng = np.random.default_rng(3)
    for _ in range(50):
        d = rng.uniform(-1.5, 1.5, 3) * h
        K = O.kernel_grad(d, h)
        Km = O.kernel_grad(-d, h)
        assert np.array_equal(Km, -K)                       # odd, bitwise
        assert np.linalg.norm(np.cross(K, d)) <= 1e-12 * (np.linalg.norm(K) * np.linalg.norm(d) + 1e-300)
        assert np.dot(K, d) <= 0.0                          # points from i towards j
    assert np.all(O.kernel_grad((2.0 * h, 0, 0), h) == 0.0)
    assert np.all(O.kernel_grad((1.5 * h, 1.5 * h, 0), h) == 0.0)
    # continuity across q = 1 and q = 2
    for q in (1.0, 2.0):
        a = O.kernel_grad(((q - 1e-9) * h, 0, 0), h)
        b = O.kernel_grad(((q + 1e-9) * h, 0, 0), h)
        assert abs(a[0] - b[0]) < 1e-7


def _poly_grid(n, h, coef):
    ax = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    a, b, c, d, e, f, g, hh, i, j = coef
    val = a + b * x + c * y + d * z + e * x * x + f * y * y + g * z * z + hh * x * y + i * y * z + j * x * z
    gx = b + 2 * e * x + hh * y + j * z
    gy = c + 2 * f * y + hh * x + i * z
    gz = d + 2 * g * z + i * y + j * x
    return val, np.stack([gx, gy, gz])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lattice_gradient_exact_for_quadratics(seed):
    n, h = 8, 0.125
    coef = np.random.default_rng(seed).uniform(-2, 2, 10)
    f, grad = _poly_grid(n, h, coef)
    D = O.lattice_gradient(f, h)
    inner = (slice(None), slice(1, n - 1), slice(1, n - 1), slice(1, n - 1))  # stencil does not wrap
    np.testing.assert_allclose(D[inner], grad[inner], rtol=0, atol=1e-11)


def test_lattice_gradient_of_constant_is_zero_bitwise():
    f = np.full((6, 5, 4), 3.7)
    assert np.all(O.lattice_gradient(f, 0.1) == 0.0)


def test_lattice_weights_sum():
    """kappa g(q)/q on the three neighbour shells: w1 + 4 w_sqrt2 + 4 w_sqrt3 = 1/2."""
    h = 1.0
    w1 = O.kernel_grad((-1, 0, 0), h)[0]
    w2 = O.kernel_grad((-1, -1, 0), h)[0]
    w3 = O.kernel_grad((-1, -1, -1), h)[0]
    assert abs(w1 + 4 * w2 + 4 * w3 - 0.5) < 1e-15
    assert w1 > w2 > w3 > 0


# ---------------------------------------------------------------- limiters
def test_limiters():
    mm, mc, vl, sb = O.LIM_MINMOD, O.LIM_MC, O.LIM_VANLEER, O.LIM_SUPERBEE
    for k in (mm, mc, vl, sb):
        assert O.limiter(k, 1.0, -2.0) == 0.0
        assert O.limiter(k, 0.0, 2.0) == 0.0
        assert O.limiter(k, 2.0, 2.0) == 2.0          # smooth data: the central slope
        assert O.limiter(k, -1.0, -3.0) == -O.limiter(k, 1.0, 3.0)
        assert O.limiter(k, 1.0, 3.0) == O.limiter(k, 3.0, 1.0)
        # Sweby's TVD region: 0 <= phi(r) <= min(2r, 2) with phi = lim(a, b)/a, r = b/a
        for r in np.linspace(0.01, 10, 57):
            phi = O.limiter(k, 1.0, r)
            assert -1e-15 <= phi <= min(2 * r, 2.0) + 1e-12
    assert O.limiter(mm, 1.0, 3.0) == 1.0
    assert O.limiter(mc, 1.0, 3.0) == 2.0
    assert O.limiter(vl, 1.0, 3.0) == 1.5
    assert O.limiter(sb, 1.0, 3.0) == 2.0
    assert O.limiter(sb, 1.0, 1.5) == 1.5


# ---------------------------------------------------------------- EOS
def test_primitive_conserved_round_trip():
    pr = P.random_state((5, 4, 6), seed=7, gamma=1.4)
    s = oracle_sim(pr)
    U = s.conserved()
    W = pr.prim
    g = pr.gamma
    np.testing.assert_array_equal(U[0], W[0])
    np.testing.assert_allclose(U[1:4], W[0] * W[1:4], rtol=1e-15)
    e = W[4] / (g - 1) + 0.5 * W[0] * np.sum(W[1:4] ** 2, axis=0)   # E = rho(|u|^2/2 + eps)
    np.testing.assert_allclose(U[4], e, rtol=1e-15)
    np.testing.assert_allclose(s.primitive(), W, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- boundary rules
def _map(idx, n, kind):
    """Source index and reflection flag of one coordinate (None: Dirichlet)."""
    if 0 <= idx < n:
        return idx, False
    if kind == P.PERIODIC:
        return idx % n, False
    if kind == P.OUTFLOW:
        return (0 if idx < 0 else n - 1), False
    if kind == P.REFLECT:
        return (-idx - 1 if idx < 0 else 2 * n - 1 - idx), True
    return None, False


@pytest.mark.parametrize("bc", [
    (P.PERIODIC,) * 6,
    (P.OUTFLOW,) * 6,
    (P.INFLOW, P.OUTFLOW, P.PERIODIC, P.PERIODIC, P.REFLECT, P.REFLECT),
    (P.REFLECT, P.INFLOW, P.OUTFLOW, P.INFLOW, P.PERIODIC, P.PERIODIC),
])
@pytest.mark.parametrize("role", [0, 1, 2, 4, 5, 7, 8])
def test_ghost_fill_rules(bc, role):
    nx, ny, nz = 4, 5, 6
    inflow = {f: (1.0 + f, 0.1 * f, -0.2, 0.3, 2.0 + f) for f in range(6)}
    s = O.OracleSim((nx, ny, nz), 0.25, gamma=1.4, bc=bc, inflow=inflow)
    g = 2
    a = np.random.default_rng(role).uniform(-1, 1, (nz + 2 * g, ny + 2 * g, nx + 2 * g))
    orig = a.copy()
    dt = 0.03
    s.fill_ghosts_padded(a, role, dt)
    n = (nx, ny, nz)
    cons = {0: lambda w: w[0], 1: lambda w: w[0] * w[1], 2: lambda w: w[0] * w[2],
            3: lambda w: w[0] * w[3],
            4: lambda w: w[4] / 0.4 + 0.5 * w[0] * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2),
            5: lambda w: dt * w[1], 6: lambda w: dt * w[2], 7: lambda w: dt * w[3]}
    for k in range(-g, nz + g):
        for j in range(-g, ny + g):
            for i in range(-g, nx + g):
                c = [i, j, k]
                sign = 1.0
                expect = None
                # the last axis filled (z) decides first
                for ax in (2, 1, 0):
                    if 0 <= c[ax] < n[ax]:
                        continue
                    face = 2 * ax + (0 if c[ax] < 0 else 1)
                    kind = bc[face]
                    if kind == P.INFLOW and role != 8:
                        expect = sign * cons[role](inflow[face])
                        break
                    src, refl = _map(c[ax], n[ax], P.OUTFLOW if kind == P.INFLOW else kind)
                    c[ax] = src
                    if refl and role in (1 + ax, 5 + ax):
                        sign = -sign
                if expect is None:
                    expect = sign * orig[c[2] + g, c[1] + g, c[0] + g]
                assert a[k + g, j + g, i + g] == pytest.approx(expect, rel=1e-15, abs=0), (i, j, k)


# ---------------------------------------------------------------- potential at r*
def test_trilinear_potential():
    nx, ny, nz = 6, 5, 7
    h = 0.2
    s = O.OracleSim((nx, ny, nz), h, bc=(P.OUTFLOW,) * 6)
    x, y, z = P.centres((nx, ny, nz), h)
    rng = np.random.default_rng(5)
    off = rng.uniform(-0.9, 0.9, (3, nz, ny, nx)) * h
    # a trilinear field is reproduced exactly on the interior (away from copied ghosts)
    a = rng.uniform(-1, 1, 8)
    f = lambda X, Y, Z: (a[0] + a[1] * X + a[2] * Y + a[3] * Z + a[4] * X * Y + a[5] * Y * Z
                         + a[6] * X * Z + a[7] * X * Y * Z)
    psi = np.ascontiguousarray(np.broadcast_to(f(x, y, z), (nz, ny, nx)))
    s.set_potential(psi)
    got = s.interp_psi(off)
    want = f(x + off[0], y + off[1], z + off[2])
    inner = (slice(1, nz - 1), slice(1, ny - 1), slice(1, nx - 1))
    np.testing.assert_allclose(got[inner], want[inner], rtol=0, atol=1e-13)
    # zero offset returns the cell value bitwise
    assert np.array_equal(s.interp_psi(np.zeros((3, nz, ny, nx))), psi)
