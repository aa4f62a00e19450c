"""Self-similar solution of the point explosion in a uniform cold gas (the
Sedov-Taylor blast wave), for checking the time-integrated Sedov runs as
the paper does (Section III-A, validation).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).  Written from the
mathematics: with the shock radius R(t) = xi0 (E t^2 / rho0)^(1/5) and
u = R' f(x), rho = rho0 g(x), p = rho0 R'^2 h(x) at x = r / R, the spherical
Euler equations (mass, momentum, and entropy p rho^-gamma constant along a
fluid path) become three ODEs in x:
    (f - x) g' + g f' + 2 f g / x = 0
    (f - x) f' - 3 f / 2 + h' / g = 0
    (f - x) (h'/h - gamma g'/g) = 3
integrated inwards from the strong-shock state at x = 1 (f = 2/(gamma+1),
g = (gamma+1)/(gamma-1), h = 2/(gamma+1)); the energy integral
E = 4 pi rho0 R'^2 R^3 int_0^1 (g f^2 / 2 + h / (gamma - 1)) x^2 dx fixes
xi0 = (25 / (16 pi I))^(1/5).  scipy's adaptive integrator and quadrature
are used as library steps.  FP64.

Pinned by ``tests/test_oracle_sedov.py`` (published xi0 for gamma = 1.4 and
5/3, the strong-shock density jump, energy and mass integrals).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.integrate import solve_ivp


def _rhs(x, y, gamma):
    f, g, h = y
    D = f - x
    a = h / g
    fp = (1.5 * f * D - a * (3.0 - 2.0 * gamma * f / x)) / (D * D - gamma * a)
    gp = -g * (fp + 2.0 * f / x) / D
    hp = h * (3.0 / D + gamma * gp / g)
    return [fp, gp, hp]


@lru_cache(maxsize=8)
def profile(gamma: float, x_min: float = 1e-4, n: int = 4001):
    """(x, f, g, h) on x in [x_min, 1] (x ascending) and xi0."""
    y1 = [2.0 / (gamma + 1.0), (gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0)]
    xs = np.linspace(1.0, x_min, n)
    sol = solve_ivp(_rhs, (1.0, x_min), y1, t_eval=xs, args=(gamma,), method="DOP853", rtol=1e-12, atol=1e-14)
    if not sol.success:
        raise RuntimeError(sol.message)
    x = sol.t[::-1]
    f, g, h = (sol.y[k][::-1] for k in range(3))
    integrand = (0.5 * g * f * f + h / (gamma - 1.0)) * x * x
    I = np.trapezoid(integrand, x)
    xi0 = (25.0 / (16.0 * math.pi * I)) ** 0.2
    return x, f, g, h, xi0


def shock_radius(E, rho0, t, gamma):
    return profile(gamma)[4] * (E * t * t / rho0) ** 0.2


def sample(r, E, rho0, t, gamma):
    """(rho, u, p) at radii r (the cold gas at rest outside the shock)."""
    x, f, g, h, xi0 = profile(gamma)
    R = xi0 * (E * t * t / rho0) ** 0.2
    Rd = 0.4 * R / t
    q = np.asarray(r, dtype=np.float64) / R
    inside = q < 1.0
    qq = np.clip(q, x[0], 1.0)
    rho = np.where(inside, rho0 * np.interp(qq, x, g), rho0)
    u = np.where(inside, Rd * np.interp(qq, x, f), 0.0)
    p = np.where(inside, rho0 * Rd * Rd * np.interp(qq, x, h), 0.0)
    return rho, u, p
