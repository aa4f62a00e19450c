"""Pins of the FP64 leapfrog step (oracle/integrate.py): free streaming,
exact momentum conservation, energy conservation to the step's order, and
second-order convergence (the error of one step against two half steps
falls as dt^3).  CPU only."""
import numpy as np
import pytest

import oracle
import sphinputs
from oracle import integrate as OI


def _case(n=600, seed=7, vel=0.3):
    ps = sphinputs.uniform(n, seed, velocity=True)
    rng = np.random.default_rng(seed)
    for k in ("vx", "vy", "vz"):
        setattr(ps, k, rng.uniform(-vel, vel, n))
    ps.u = rng.uniform(1.0, 2.0, n)          # pressure gradients: non-zero forces
    h = np.asarray(ps.h0, dtype=np.float64) * 1.1
    return ps, h


def _state(r):
    return np.concatenate([r["x"], r["y"], r["z"], r["vx"], r["vy"], r["vz"], r["u"]])


def _advance(ps, r):
    q = sphinputs.ParticleSet(r["x"], r["y"], r["z"], ps.m, r["u"], r["vx"], r["vy"], r["vz"], ps.h0, ps.box)
    return q


def test_uniform_flow_streams_freely():
    ps = sphinputs.lattice(8, 0.0, 1)
    w = (0.3, -0.2, 0.1)
    ps.vx, ps.vy, ps.vz = (np.full(ps.n, c) for c in w)
    h = np.asarray(ps.h0, dtype=np.float64)
    r = OI.kdk_step(ps, h, 0.01)
    for k, c in zip(("x", "y", "z"), w):
        assert np.allclose(r[k], (getattr(ps, k) + 0.01 * c) % 1.0, atol=1e-12)
    for k, c in zip(("vx", "vy", "vz"), w):
        assert np.allclose(r[k], c, atol=1e-12)
    assert np.allclose(r["u"], ps.u, atol=1e-12)


def test_momentum_conserved_exactly_and_energy_to_order():
    ps, h = _case()
    m = np.asarray(ps.m)
    f = OI.kdk_step(ps, h, 1e-9)["f0"]
    dt = 0.3 * float(np.min(h / f["vsig"]))
    r = OI.kdk_step(ps, h, dt)
    p0 = [np.sum(m * getattr(ps, k)) for k in ("vx", "vy", "vz")]
    p1 = [np.sum(m * r[k]) for k in ("vx", "vy", "vz")]
    pscale = np.sum(m * np.abs(ps.vx))
    assert np.allclose(p0, p1, atol=1e-13 * pscale + 1e-15)
    e0 = np.sum(m * (0.5 * (ps.vx ** 2 + ps.vy ** 2 + ps.vz ** 2) + ps.u))
    e1 = np.sum(m * (0.5 * (r["vx"] ** 2 + r["vy"] ** 2 + r["vz"] ** 2) + r["u"]))
    # energy is not exact for a finite step, but far below the first-order
    # change dt * sum m |v.a + du/dt|
    first = dt * np.sum(m * np.abs(ps.vx * r["f0"]["ax"] + ps.vy * r["f0"]["ay"] + ps.vz * r["f0"]["az"]
                                   + r["f0"]["dudt"]))
    assert abs(e1 - e0) < 0.05 * first


def test_second_order():
    ps, h = _case()
    f = OI.kdk_step(ps, h, 1e-9)["f0"]
    dt0 = 0.3 * float(np.min(h / f["vsig"]))
    errs = []
    for dt in (dt0, 0.5 * dt0):
        one = OI.kdk_step(ps, h, 2 * dt)
        half = OI.kdk_step(ps, h, dt)
        two = OI.kdk_step(_advance(ps, half), h, dt)
        d = _state(one) - _state(two)
        n = ps.n
        d[: 3 * n] = (d[: 3 * n] + 0.5) % 1.0 - 0.5     # periodic positions
        errs.append(np.abs(d).max())
    # local error of a second-order step: O(dt^3), so halving dt divides it by ~8
    assert errs[0] / errs[1] > 5.0, errs
