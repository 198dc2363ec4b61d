"""Sedov-Taylor point blast: the similarity solution of a strong spherical shock
(test-side reference, independent of the scheme).

A point explosion of energy E in a gas of density rho0 and negligible pressure
drives a shock of radius R = xi0 (E t^2 / rho0)^(1/5).  With eta = r/R and
u = R' f(eta), rho = rho0 g(eta), p = rho0 R'^2 h(eta) (R' = dR/dt = 2R/5t), the
spherical Euler equations become ordinary differential equations in eta:
  continuity  (f - eta) g' + g f' + 2 g f / eta = 0
  momentum    (f - eta) f' + h'/g = 3 f / 2
  entropy     (f - eta) (h'/h - gamma g'/g) = 3
with the strong-shock jump conditions at eta = 1:
  f = 2/(gamma+1), g = (gamma+1)/(gamma-1), h = 2/(gamma+1).
They are integrated from the shock inwards; the energy inside the shock,
E = rho0 R'^2 R^3 I with I = int_0^1 (g f^2/2 + h/(gamma-1)) 4 pi eta^2 d eta, then
fixes xi0 = (25 / (4 I))^(1/5).
"""
import math

import numpy as np


def _rhs(eta, y, gamma):
    f, g, h = y
    d = f - eta
    # eliminate g' and h' (continuity, entropy) from the momentum equation
    num = 1.5 * f * d - (h / g) * (3.0 - 2.0 * gamma * f / eta)
    den = d * d - gamma * h / g
    fp = num / den
    gp = -g * (fp + 2.0 * f / eta) / d
    hp = h * (3.0 / d + gamma * gp / g)
    return [fp, gp, hp]


def profile(gamma, eta_min=1e-3, n=4001):
    """f, g, h on eta in [eta_min, 1] (the solution near the centre carries a
    vanishing share of the mass and energy)."""
    from scipy.integrate import solve_ivp
    y1 = [2.0 / (gamma + 1.0), (gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0)]
    eta = np.linspace(1.0, eta_min, n)
    sol = solve_ivp(_rhs, (1.0, eta_min), y1, t_eval=eta, args=(gamma,), rtol=1e-10, atol=1e-12,
                    method="LSODA")
    assert sol.success, sol.message
    return sol.t[::-1], sol.y[:, ::-1]


def xi0(gamma):
    """The constant of R = xi0 (E t^2 / rho0)^(1/5)."""
    eta, (f, g, h) = profile(gamma)
    integrand = (0.5 * g * f * f + h / (gamma - 1.0)) * 4.0 * math.pi * eta * eta
    I = float(np.trapezoid(integrand, eta))
    return (25.0 / (4.0 * I)) ** 0.2


def radius(t, gamma, energy=1.0, rho0=1.0):
    return xi0(gamma) * (energy * t * t / rho0) ** 0.2


def mass_fraction(gamma):
    """Mass inside the shock over the swept mass (4/3) pi R^3 rho0: 1 for the exact
    solution (a check of the integration)."""
    eta, (f, g, h) = profile(gamma)
    return float(np.trapezoid(g * 3.0 * eta * eta, eta))
