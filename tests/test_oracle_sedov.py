"""Pins of the Sedov-Taylor solution (oracle/sedov.py): the published
energy constant for two adiabatic indices, mass conservation of the
profile, and its centre and shock limits.  CPU only."""
import os

import numpy as np
import pytest

from oracle import sedov as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sedov_alpha.txt")


def _rows():
    return [line.split() for line in open(GOLD) if line.strip() and not line.startswith("#")]


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"gamma{float(r[0]):.3f}")
def test_energy_constant_matches_published_value(row):
    g, printed = float(row[0]), row[1]
    alpha = S.profile(g)[4] ** -5
    dec = len(printed.split(".")[1])
    assert abs(alpha - float(printed)) <= 0.5 * 10.0 ** -dec, alpha


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0, 1.2])
def test_swept_mass_is_in_the_shell(g):
    """The gas inside the shock is all the gas it has swept: int g x^2 dx = 1/3."""
    x, f, gg, h, _ = S.profile(g)
    assert np.trapezoid(gg * x * x, x) == pytest.approx(1.0 / 3.0, rel=1e-5)


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_limits(g):
    x, f, gg, h, _ = S.profile(g)
    # strong-shock state behind the front
    assert gg[-1] == pytest.approx((g + 1) / (g - 1)) and f[-1] == pytest.approx(2 / (g + 1))
    # centre: empty, finite pressure, homologous flow u ~ r / (gamma t) (f / x -> 1/gamma)
    assert gg[0] < 1e-10 and h[0] > 0.1 * h[-1]
    assert f[1] / x[1] == pytest.approx(1.0 / g, rel=0.03)
    # density rises and velocity grows monotonically out to the shock
    assert np.all(np.diff(gg) > 0) and np.all(np.diff(f) > 0)


def test_sample_and_radius():
    E, rho0, t, g = 100.0, 1.0, 5e-3, 5.0 / 3.0
    R = S.shock_radius(E, rho0, t, g)
    assert R == pytest.approx(S.profile(g)[4] * (E * t * t) ** 0.2)
    rho, u, p = S.sample(np.array([0.5 * R, 0.99999 * R, 1.001 * R]), E, rho0, t, g)
    assert rho[2] == rho0 and u[2] == 0.0 and p[2] == 0.0
    assert rho[1] == pytest.approx(4.0, rel=0.01) and u[1] == pytest.approx(0.75 * 0.4 * R / t, rel=0.01)
    # energy in the blast equals E
    r = np.linspace(1e-6, R * (1 - 1e-9), 200001)
    rho, u, p = S.sample(r, E, rho0, t, g)
    e = np.trapezoid((0.5 * rho * u * u + p / (g - 1)) * 4 * np.pi * r * r, r)
    assert e == pytest.approx(E, rel=1e-3)
