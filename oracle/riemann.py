"""Exact solution of the Riemann problem of an ideal gas (1-D Euler
equations), for checking the time-integrated shock-tube runs against the
analytic result, as the paper does for its Sod-shock test (Section III-A,
validation).

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).  Written from the
textbook mathematics of the exact solver (the star-region pressure is the
root of f_L(p) + f_R(p) + (u_R - u_L) = 0, with f_K the shock
(Rankine-Hugoniot) or rarefaction (isentropic, Riemann invariant) branch;
the solution is self-similar in x/t).  FP64 throughout.

Pinned by ``tests/test_oracle_riemann.py``: published star states of three
standard test problems, and the jump and invariant conditions that every
sampled solution must satisfy.
"""
from __future__ import annotations

import math

import numpy as np


def _branch(p, rho, pk, gamma):
    """f_K(p) and its derivative for the side with state (rho, pk)."""
    a = math.sqrt(gamma * pk / rho)
    if p > pk:   # shock: Rankine-Hugoniot
        A = 2.0 / ((gamma + 1.0) * rho)
        Bk = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(A / (p + Bk))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + Bk))
    # rarefaction: isentropic, along the Riemann invariant
    r = (p / pk) ** ((gamma - 1.0) / (2.0 * gamma))
    return 2.0 * a / (gamma - 1.0) * (r - 1.0), (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * a)


def star(rhoL, uL, pL, rhoR, uR, pR, gamma):
    """(p*, u*) of the star region (Newton iteration on the pressure)."""
    aL, aR = math.sqrt(gamma * pL / rhoL), math.sqrt(gamma * pR / rhoR)
    if 2.0 * (aL + aR) / (gamma - 1.0) <= uR - uL:
        raise ValueError("the data generate vacuum")
    # two-rarefaction estimate as the starting point (positive by construction)
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((aL + aR - 0.5 * (gamma - 1.0) * (uR - uL)) / (aL / pL ** z + aR / pR ** z)) ** (1.0 / z)
    for _ in range(100):
        fL, dL = _branch(p, rhoL, pL, gamma)
        fR, dR = _branch(p, rhoR, pR, gamma)
        step = (fL + fR + uR - uL) / (dL + dR)
        pn = max(p - step, 1e-14 * p)
        done = abs(pn - p) <= 1e-15 * (pn + p)
        p = pn
        if done:
            break
    fL, _ = _branch(p, rhoL, pL, gamma)
    fR, _ = _branch(p, rhoR, pR, gamma)
    return p, 0.5 * (uL + uR) + 0.5 * (fR - fL)


def sample(xi, rhoL, uL, pL, rhoR, uR, pR, gamma):
    """(rho, u, p) at the self-similar coordinate xi = (x - x0) / t (arrays)."""
    xi = np.asarray(xi, dtype=np.float64)
    ps, us = star(rhoL, uL, pL, rhoR, uR, pR, gamma)
    g1, g2 = (gamma - 1.0) / (gamma + 1.0), (gamma - 1.0) / (2.0 * gamma)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for side, (rk, uk, pk) in (("L", (rhoL, uL, pL)), ("R", (rhoR, uR, pR))):
        ak = math.sqrt(gamma * pk / rk)
        s = 1.0 if side == "R" else -1.0        # the wave moves towards +s
        on = xi > us if side == "R" else xi <= us
        x = xi[on]
        r = np.empty_like(x)
        v = np.empty_like(x)
        q = np.empty_like(x)
        if ps > pk:   # shock of speed uk + s ak sqrt(...)
            S = uk + s * ak * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pk + g2)
            outside = s * (x - S) >= 0.0
            rs = rk * (ps / pk + g1) / (g1 * ps / pk + 1.0)
            r[:], v[:], q[:] = rs, us, ps
        else:         # rarefaction between head and tail
            head = uk + s * ak
            astar = ak * (ps / pk) ** g2
            tail = us + s * astar
            outside = s * (x - head) >= 0.0
            rs = rk * (ps / pk) ** (1.0 / gamma)
            r[:], v[:], q[:] = rs, us, ps
            fan = (~outside) & (s * (x - tail) > 0.0)
            xf = x[fan]
            c = 2.0 / (gamma + 1.0) * (ak - s * 0.5 * (gamma - 1.0) * (uk - xf))
            v[fan] = 2.0 / (gamma + 1.0) * (-s * ak + 0.5 * (gamma - 1.0) * uk + xf)
            r[fan] = rk * (c / ak) ** (2.0 / (gamma - 1.0))
            q[fan] = pk * (c / ak) ** (2.0 * gamma / (gamma - 1.0))
        r[outside], v[outside], q[outside] = rk, uk, pk
        rho[on], u[on], p[on] = r, v, q
    return rho, u, p
