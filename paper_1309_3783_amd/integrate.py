"""Time stepping of a batch over the C-ABI: kick-drift-kick leapfrog with one
step for all particles and every force recomputed each step, as in the
paper's validation runs (Section III-A).  Argument marshalling only: the
kicks, drifts, Courant minimum, cell build, h solve and forces all run in
the library's kernels.

One step of size dt, from positions x_n, velocities v_n, energies u_n and
the forces a_n, du_n computed at them:
  v_h = v_n + dt/2 a_n,  u_h = u_n + dt/2 du_n          (kick)
  x_{n+1} = x_n + dt v_h  (wrapped into the box)        (drift)
  v_p = v_h + dt/2 a_n,  u_p = u_h + dt/2 du_n          (prediction)
  a_{n+1}, du_{n+1} at (x_{n+1}, v_p, u_p), h solved from h_n
  v_{n+1} = v_h + dt/2 a_{n+1},  u_{n+1} = u_h + dt/2 du_{n+1}  (kick)
The prediction gives the viscosity and the pressure of the new forces the
velocities and energies of the end of the step.
"""
from __future__ import annotations

import dataclasses

from . import binding as B


class Leapfrog:
    """State of one batch under time integration (device tensors, caller
    order).  The batch's x, y, z, vx, vy, vz, u are advanced in place."""

    def __init__(self, ctx: B.Context, batch: B.Batch, prm=None, c_cfl: float = 0.3, solve_h: bool = True,
                 reuse: bool = False):
        """solve_h False: the smoothing lengths stay at batch.h (density
        without the Newton solve), as in a comparison at fixed h.
        reuse: keep the cells and sorted lists from step to step while they
        still cover the moved particles (sph_refresh_cells), building them
        again only when the library refuses the refresh or h outgrows them."""
        import torch
        self.ctx, self.b = ctx, batch
        self.prm = prm or B.params()
        self.c_cfl = float(c_cfl)
        self.solve = solve_h
        self.reuse = reuse
        self.tree = B.Tree(ctx)
        self.d = B.DensityOut(batch.n, batch.x.device)
        self.f = B.ForceOut(batch.n, batch.nsets, batch.x.device)
        self.vp = tuple(torch.empty_like(batch.vx) for _ in range(3))
        self.up = torch.empty_like(batch.u)
        self.t = 0.0
        self.steps = 0
        self.newton_iterations = 0
        self._forces(batch.vx, batch.vy, batch.vz, batch.u, batch.h)

    def _forces(self, vx, vy, vz, u, h):
        view = dataclasses.replace(self.b, vx=vx, vy=vy, vz=vz, u=u, h=h, keep=[])
        if self.solve:
            st, nu, it = B.solve_with_rebuild(self.tree, view, self.prm, self.d, refresh=self.reuse)
            if st not in (B.SPH_OK, B.SPH_E_NOCONV):
                raise B.SphError(st, "solve_h during time integration")
            self.newton_iterations += it
        else:
            if not (self.reuse and self.tree.same_layout(view) and self.tree.refresh(view)):
                self.tree.build_cells(view, self.prm)
                self.tree.sort_pairs()
            self.tree.density(self.d)
        self.tree.force(self.f)

    def cfl_dt(self) -> float:
        """c_cfl min_i h_i / vsig_i at the current forces."""
        return B.cfl_dt(self.ctx, self.d.h, self.f.vsig, self.c_cfl)

    def step(self, dt: float):
        b, f, ctx = self.b, self.f, self.ctx
        v = (b.vx, b.vy, b.vz)
        a = (f.ax, f.ay, f.az)
        B.kick(ctx, 0.5 * dt, v, b.u, a, f.dudt)
        B.drift(ctx, b, dt)
        B.kick(ctx, 0.5 * dt, v, b.u, a, f.dudt, v_out=self.vp, u_out=self.up)
        self._forces(*self.vp, self.up, self.d.h.clone() if self.solve else self.b.h)
        B.kick(ctx, 0.5 * dt, v, b.u, (f.ax, f.ay, f.az), f.dudt)
        self.t += dt
        self.steps += 1

    def run(self, t_end: float, dt: float | None = None, max_steps: int = 100000) -> int:
        """Advance to t_end with the fixed step dt, or (dt None) with the
        Courant step of the current forces, one for all particles, each step;
        the last step is shortened to end at t_end.  Returns the steps taken."""
        k = 0
        while self.t < t_end * (1 - 1e-12) and k < max_steps:
            h = dt if dt is not None else self.cfl_dt()
            h = min(h, t_end - self.t)
            self.step(h)
            k += 1
        return k

    def energy(self) -> float:
        """Total energy sum m (v^2/2 + u) (FP64, on the host)."""
        b = self.b
        m = b.m.double()
        ke = 0.5 * (b.vx.double() ** 2 + b.vy.double() ** 2 + b.vz.double() ** 2)
        return float((m * (ke + b.u.double())).sum())

    def momentum(self):
        b = self.b
        m = b.m.double()
        return tuple(float((m * v.double()).sum()) for v in (b.vx, b.vy, b.vz))
