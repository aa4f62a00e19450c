"""Test-side input preparation shared by the GPU parity tests and the bench.

Inputs come from ``sphinputs`` (seeded generators).  Smoothing lengths for
the fixed-h protocol come from the FP64 oracle (never from the GPU path):
solved to 1e-9 in N_w, rounded to FP32, then nudged so that no pair lies
within 1e-6 (relative) of either particle's cutoff -- the membership of such
a pair in the density or force set would hinge on FP32 rounding.
"""
import numpy as np

import oracle
import sphinputs

TIE_REL = 1e-6
TIE_BUMP = 3e-6


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def untie_h(ps, h, rel=TIE_REL, max_rounds=50):
    """Raise h (FP32 steps) of particles with a pair near a cutoff until none is."""
    h = f32(h).copy()
    bumped = 0
    for _ in range(max_rounds):
        bad = oracle.near_cutoff(ps.x, ps.y, ps.z, h, ps.box, rel=rel)
        if not bad.any():
            return h, bumped
        bumped += int(bad.sum())
        h[bad] = f32(h[bad] * (1.0 + TIE_BUMP))
    raise RuntimeError("could not separate pairs from cutoffs")


def redraw_ties_uniform(ps, h, seed, rel=TIE_REL, max_rounds=50):
    """Constant-h uniform set: redraw particles that have a pair near the cutoff."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(max_rounds):
        bad = oracle.near_cutoff(ps.x, ps.y, ps.z, h, ps.box, rel=rel)
        if not bad.any():
            return ps
        idx = np.nonzero(bad)[0]
        new = np.floor(rng.random((idx.size, 3)) * sphinputs.GRID) / sphinputs.GRID
        ps.x[idx], ps.y[idx], ps.z[idx] = new[:, 0], new[:, 1], new[:, 2]
        k = np.round(ps.pos() * sphinputs.GRID).astype(np.int64)
        _, first = np.unique(k, axis=0, return_index=True)
        if first.size != ps.n:
            continue
    raise RuntimeError("could not separate pairs from the cutoff")


def solved_h(ps, tol=1e-9):
    h, _ = oracle.solve_h(ps.x, ps.y, ps.z, ps.m, ps.h0, ps.box, tol=tol)
    return h


def fixed_h_case(ps, h=None):
    """(ps, h) with h from the oracle solve (or given), FP32 and untied."""
    if h is None:
        h = solved_h(ps)
    h, _ = untie_h(ps, h)
    return ps, h


def cfg_small_uniform(velocity=False):
    """N = 4096 uniform, constant h for 48 expected neighbours."""
    ps = sphinputs.uniform(4096, 1, velocity=velocity)
    h = f32(np.full(ps.n, sphinputs.h_for_density(float(ps.n))))
    ps = redraw_ties_uniform(ps, h, seed=101)
    ps.h0 = h.copy()
    return ps, h


def oracle_reference(ps, h, targets=None, alpha=oracle.ALPHA):
    """Oracle density and force at fixed h (force needs rho of the neighbours,
    so the density is computed for every particle)."""
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m, ps.box)
    f = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, d["rho"], d["drho_dh"], ps.box,
                     alpha=alpha, targets=targets)
    return d, f
