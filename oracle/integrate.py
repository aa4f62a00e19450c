"""FP64 reference of one time step of the integration path: a kick-drift-kick
leapfrog with one step dt for all particles and every force recomputed at
the new positions (the paper's test runs: one fixed time step, all forces
updated each step, Section III-A; the paper does not name the integrator,
the leapfrog is this path's reading).  The force at the end of the step
takes the velocities and energies predicted for that time.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).  The smoothing
lengths are held fixed over the step (given by the caller), so that the
GPU path can be compared with it element by element.  Uses the oracle's
density and force stages; the step itself is the leapfrog written out.
"""
from __future__ import annotations

import numpy as np

from . import density, force, GAMMA, ALPHA


def _forces(x, y, z, h, m, vx, vy, vz, u, box, gamma, alpha):
    d = density(x, y, z, h, m, box)
    return force(x, y, z, h, m, vx, vy, vz, u, d["rho"], d["drho_dh"], box, gamma=gamma, alpha=alpha)


def kdk_step(ps, h, dt, gamma=GAMMA, alpha=ALPHA):
    """One step of size dt from the state of ps (positions, velocities,
    energies) at fixed h.  Returns the new state and the forces at both
    ends (dict of FP64 arrays)."""
    box = ps.box
    x, y, z = (np.asarray(a, dtype=np.float64) for a in (ps.x, ps.y, ps.z))
    v = [np.asarray(a, dtype=np.float64) for a in (ps.vx, ps.vy, ps.vz)]
    u = np.asarray(ps.u, dtype=np.float64)
    m = np.asarray(ps.m, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    f0 = _forces(x, y, z, h, m, *v, u, box, gamma, alpha)
    a0 = [f0["ax"], f0["ay"], f0["az"]]
    # kick by dt/2 with the forces at the start
    vh = [v[k] + 0.5 * dt * a0[k] for k in range(3)]
    uh = u + 0.5 * dt * f0["dudt"]
    # drift by dt, periodic wrap
    x1, y1, z1 = ((c + dt * vh[k]) % box for k, c in enumerate((x, y, z)))
    # velocities and energies predicted for the end of the step
    vp = [vh[k] + 0.5 * dt * a0[k] for k in range(3)]
    up = uh + 0.5 * dt * f0["dudt"]
    f1 = _forces(x1, y1, z1, h, m, *vp, up, box, gamma, alpha)
    a1 = [f1["ax"], f1["ay"], f1["az"]]
    # kick by dt/2 with the forces at the end
    v1 = [vh[k] + 0.5 * dt * a1[k] for k in range(3)]
    u1 = uh + 0.5 * dt * f1["dudt"]
    return {"x": x1, "y": y1, "z": z1, "vx": v1[0], "vy": v1[1], "vz": v1[2], "u": u1,
            "f0": f0, "f1": f1}
