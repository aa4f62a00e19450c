"""Seeded synthetic particle sets for the SPH density/force path.

This module only draws inputs: positions, masses, internal energies,
velocities and a first guess of the smoothing length taken from the
analytic number density of each sampling recipe.  It holds none of the
SPH arithmetic (no kernel, no neighbour sums) so that both the FP64 oracle
and the GPU path can take their inputs from here without sharing method
code.

By default every position is snapped to the 2^-24 grid of the periodic unit
cube and exact duplicates are redrawn, so that any coordinate difference
between two particles of one top-level cell is exactly representable in
FP32.  With ``snap=False`` the positions keep all their FP64 bits (wrapped
into [0, 1)): the off-grid inputs a caller or a time step produces.

Recipes (all periodic unit box, equal masses m = FP32(1/N), u = 1.5):

* ``uniform``   -- N uniform points (the small constant-h case).
* ``lattice``   -- simple-cubic lattice of n^3 points, spacing 1/n, each
                   coordinate jittered by U(-j, +j) spacings (j = 0: perfect).
                   Stands in for the Sedov-blast lattice of Section III-B.
* ``sod``       -- the shock tube of the paper's validation runs (Section
                   III-A): a dense half x < 1/2 (density 1, pressure 1) and a
                   light half (density ~1/4, pressure 0.1795) of equal-mass
                   particles on two simple-cubic lattices, at rest; u from the
                   ideal-gas law (gamma = 5/3).  Its default sizes (780,448 +
                   197,173 particles) stand in for the paper's 800,000 +
                   200,000.
* ``sedov``     -- the blast of the paper's validation runs (Section III-A):
                   a simple-cubic lattice at rest with density 1 and pressure
                   1e-5, the energy E = 100 given to the 33 particles nearest
                   the centre (u = E / 33 / m each).
* ``plummer_mixture`` -- 64 Plummer spheres (scale radius a = 10^U(-3,-1),
                   truncated at min(20a, 0.45)) holding 80% of the particles
                   plus a 20% uniform background.  Stands in for the
                   cosmological volume of Section III-B (its data are not
                   available), reproducing its ~3 decades of smoothing length.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GRID = float(2 ** 24)          # positions live on k * 2^-24
N_NGB = 48.0                   # target neighbour number (Section III-B constants)
U_DEFAULT = 1.5                # uniform internal energy: P = rho for gamma = 5/3


@dataclass
class ParticleSet:
    """One particle set in caller order (FP64 positions, FP32-exact scalars)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    u: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    h0: np.ndarray              # first guess of h (FP32-exact)
    box: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def pos(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _f32(a) -> np.ndarray:
    """Round to the nearest FP32 value, returned as FP64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _snap_unique(pos: np.ndarray, redraw, rng: np.random.Generator, snap: bool = True) -> np.ndarray:
    """Snap positions to the 2^-24 grid (mod 1) and redraw exact duplicates;
    snap=False: wrap into [0, 1) only, redrawing positions whose 2^-24 cell
    is taken (distinct particles stay at least ~2^-24 apart either way)."""
    for _ in range(64):
        w = np.mod(pos, 1.0)
        k = np.floor(w * GRID).astype(np.int64) % int(GRID)
        dup = _duplicates(k)
        if not dup.any():
            return k.astype(np.float64) / GRID if snap else w
        idx = np.nonzero(dup)[0]
        pos = pos.copy()
        pos[idx] = redraw(idx, rng)
    raise RuntimeError("could not draw unique positions")


def _duplicates(k: np.ndarray) -> np.ndarray:
    """Mask of rows of k (integer triples) equal to an earlier row in sort
    order (every duplicate but one)."""
    order = np.lexsort((k[:, 2], k[:, 1], k[:, 0]))
    ks = k[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    dup = np.zeros(k.shape[0], dtype=bool)
    dup[order[1:][same]] = True
    return dup


def _finish(pos, n, rng, h0, velocity, meta) -> ParticleSet:
    m = np.full(n, float(np.float32(1.0 / n)))
    u = np.full(n, U_DEFAULT)
    if velocity:
        v = _f32(rng.uniform(-0.1, 0.1, size=(n, 3)))
    else:
        v = np.zeros((n, 3))
    return ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(),
                       m, u, v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(),
                       _f32(h0), 1.0, meta)


def h_for_density(n_density, n_ngb: float = N_NGB) -> np.ndarray:
    """Radius of a sphere holding n_ngb points at number density n_density."""
    return np.cbrt(3.0 * n_ngb / (4.0 * math.pi * np.asarray(n_density, dtype=np.float64)))


def uniform(n: int, seed: int, velocity: bool = False, snap: bool = True) -> ParticleSet:
    rng = _rng(seed)
    pos = rng.random((n, 3))
    pos = _snap_unique(pos, lambda idx, r: r.random((idx.size, 3)), rng, snap)
    h = h_for_density(float(n))
    return _finish(pos, n, rng, np.full(n, h), velocity,
                   {"recipe": "uniform", "seed": seed, "snap": snap})


def lattice(n_side: int, jitter: float, seed: int, velocity: bool = False, snap: bool = True) -> ParticleSet:
    rng = _rng(seed)
    d = 1.0 / n_side
    g = (np.arange(n_side) + 0.5) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    base = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    n = base.shape[0]
    if jitter > 0:
        pos = base + rng.uniform(-jitter, jitter, size=(n, 3)) * d
    else:
        pos = base

    def redraw(idx, r):
        return base[idx] + r.uniform(-jitter, jitter, size=(idx.size, 3)) * d

    pos = _snap_unique(pos, redraw, rng, snap)
    return _finish(pos, n, rng, np.full(n, h_for_density(float(n))), velocity,
                   {"recipe": "lattice", "n_side": n_side, "jitter": jitter, "seed": seed, "snap": snap})


def sod(n_left: int = 116, n_right: int = 73, nx_right: int = 37, p_left: float = 1.0, p_right: float = 0.1795,
        gamma: float = 5.0 / 3.0) -> ParticleSet:
    """Shock tube in the periodic unit cube: x < 1/2 holds an n_left/2 x
    n_left x n_left lattice (spacing 1/n_left, density 1), x >= 1/2 an
    nx_right x n_right x n_right lattice (spacings 1/(2 nx_right) along x,
    1/n_right across).  Equal masses; both halves at rest with the given
    pressures, u = P / ((gamma - 1) rho) from the lattice densities.  The
    tube has two interfaces (x = 0 and x = 1/2, periodic): the waves of the
    one at 1/2 stay inside [1/4, 3/4] until t ~ 0.15."""
    if n_left % 2:
        raise ValueError("n_left must be even")
    gl = (np.arange(n_left) + 0.5) / n_left
    X, Y, Z = np.meshgrid(gl[: n_left // 2], gl, gl, indexing="ij")
    left = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    gx = 0.5 + (np.arange(nx_right) + 0.5) * (0.5 / nx_right)
    gr = (np.arange(n_right) + 0.5) / n_right
    X, Y, Z = np.meshgrid(gx, gr, gr, indexing="ij")
    right = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pos = np.concatenate([left, right])
    rng = _rng(0)
    pos = _snap_unique(pos, lambda idx, r: pos[idx], rng)
    nl, nr = left.shape[0], right.shape[0]
    m = float(np.float32(0.5 / nl))                  # density 1 on the left
    rho_l, rho_r = m * nl / 0.5, m * nr / 0.5
    u = np.concatenate([np.full(nl, p_left / ((gamma - 1.0) * rho_l)),
                        np.full(nr, p_right / ((gamma - 1.0) * rho_r))])
    h0 = np.concatenate([np.full(nl, h_for_density(nl / 0.5)), np.full(nr, h_for_density(nr / 0.5))])
    n = nl + nr
    z = np.zeros(n)
    return ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, m), _f32(u),
                       z.copy(), z.copy(), z.copy(), _f32(h0), 1.0,
                       {"recipe": "sod", "n_left": nl, "n_right": nr, "rho_left": rho_l, "rho_right": rho_r,
                        "p_left": p_left, "p_right": p_right, "gamma": gamma})


def sedov(n_side: int = 101, e_total: float = 100.0, n_hot: int = 33, p0: float = 1e-5,
          gamma: float = 5.0 / 3.0) -> ParticleSet:
    """n_side^3 lattice (spacing 1/n_side, density 1) in the periodic unit
    cube, at rest with pressure p0; the n_hot particles nearest the centre
    (ties of distance broken by index) share e_total equally as internal
    energy.  With an odd n_side a lattice point sits at the centre and the
    33 nearest are the centre, its 6 face, 12 edge and 8 corner neighbours
    and the 6 points two spacings out along the axes."""
    d = 1.0 / n_side
    g = (np.arange(n_side) + 0.5) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pos = _snap_unique(pos, lambda idx, r: pos[idx], _rng(0))
    n = pos.shape[0]
    m = float(np.float32(1.0 / n))
    r2 = np.sum((pos - 0.5) ** 2, axis=1)
    hot = np.argsort(r2, kind="stable")[:n_hot]
    u = np.full(n, p0 / ((gamma - 1.0) * 1.0))
    u[hot] = e_total / n_hot / m
    z = np.zeros(n)
    return ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, m), _f32(u),
                       z.copy(), z.copy(), z.copy(), _f32(np.full(n, h_for_density(float(n)))), 1.0,
                       {"recipe": "sedov", "n_side": n_side, "e_total": e_total, "n_hot": n_hot, "p0": p0,
                        "gamma": gamma, "hot": hot})


def _plummer_radius(rng, a, rmax, size):
    umax = rmax ** 3 / (rmax ** 2 + a ** 2) ** 1.5
    u = rng.uniform(0.0, umax, size=size)
    u = np.maximum(u, 1e-300)
    return a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)


def _iso(rng, size):
    v = rng.normal(size=(size, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def plummer_mixture(n: int, seed: int, n_clumps: int = 64, bg_frac: float = 0.2,
                    velocity: bool = False, snap: bool = True) -> ParticleSet:
    rng = _rng(seed)
    n_bg = int(round(bg_frac * n))
    n_cl = n - n_bg
    per = np.full(n_clumps, n_cl // n_clumps, dtype=np.int64)
    per[: n_cl - per.sum()] += 1
    a = 10.0 ** rng.uniform(-3.0, -1.0, size=n_clumps)
    rmax = np.minimum(20.0 * a, 0.45)
    centre = rng.random((n_clumps, 3))
    parts = [rng.random((n_bg, 3))]
    owner = [np.full(n_bg, -1, dtype=np.int64)]
    for c in range(n_clumps):
        r = _plummer_radius(rng, a[c], rmax[c], per[c])
        parts.append(centre[c] + r[:, None] * _iso(rng, per[c]))
        owner.append(np.full(per[c], c, dtype=np.int64))
    pos = np.concatenate(parts, axis=0)
    own = np.concatenate(owner)

    def redraw(idx, r):
        out = np.empty((idx.size, 3))
        for k, i in enumerate(idx):
            c = own[i]
            if c < 0:
                out[k] = r.random(3)
            else:
                rr = _plummer_radius(r, a[c], rmax[c], 1)
                out[k] = centre[c] + rr[:, None] * _iso(r, 1)
        return out

    pos = _snap_unique(pos, redraw, rng, snap)
    dens = plummer_number_density(pos, n_bg, per, a, rmax, centre)
    h0 = h_for_density(dens)
    return _finish(pos, n, rng, h0, velocity,
                   {"recipe": "plummer_mixture", "seed": seed, "n_clumps": n_clumps,
                    "bg_frac": bg_frac, "a": a.tolist(), "centre": centre.tolist(), "snap": snap})


def clump_by_face(n_bg: int, n_clump: int, seed: int, radius: float = 0.03,
                  centre=(0.535, 0.375, 0.375), velocity: bool = False, snap: bool = True) -> ParticleSet:
    """A uniform background of n_bg particles and one uniform ball of
    n_clump particles just past the plane x = 1/2, which is a face of the
    top cells for every power-of-two top grid: the sparse cells on the other
    side of that plane reach the whole ball (densities differ by the ratio
    of the two number densities, h by its cube root)."""
    rng = _rng(seed)
    c = np.asarray(centre, dtype=np.float64)

    def ball(k, r):
        rr = radius * np.cbrt(r.random(k))
        return c + rr[:, None] * _iso(r, k)

    pos = np.concatenate([rng.random((n_bg, 3)), ball(n_clump, rng)], axis=0)
    is_bg = np.arange(n_bg + n_clump) < n_bg

    def redraw(idx, r):
        out = np.empty((idx.size, 3))
        nb = int(is_bg[idx].sum())
        out[is_bg[idx]] = r.random((nb, 3))
        out[~is_bg[idx]] = ball(idx.size - nb, r)
        return out

    pos = _snap_unique(pos, redraw, rng, snap)
    dens = np.full(n_bg + n_clump, float(n_bg))
    dens[~is_bg] += n_clump / (4.0 / 3.0 * math.pi * radius ** 3)
    return _finish(pos, n_bg + n_clump, rng, h_for_density(dens), velocity,
                   {"recipe": "clump_by_face", "seed": seed, "n_bg": n_bg, "n_clump": n_clump,
                    "radius": radius, "centre": list(centre), "snap": snap})


def plummer_number_density(pos, n_bg, per, a, rmax, centre):
    """Analytic number density of the truncated-Plummer mixture at ``pos``
    (each clump contributes only inside its truncation radius, so only the
    particles in the periodic x-slab around its centre are visited)."""
    out = np.full(pos.shape[0], float(n_bg))
    umax = rmax ** 3 / (rmax ** 2 + a ** 2) ** 1.5
    xs_order = np.argsort(pos[:, 0], kind="stable")
    xs = pos[xs_order, 0]
    for c in range(len(a)):
        lo, hi = centre[c, 0] - rmax[c], centre[c, 0] + rmax[c]
        spans = []
        for sh in (-1.0, 0.0, 1.0):
            a0, b0 = max(lo + sh, 0.0), min(hi + sh, 1.0)
            if a0 < b0:
                spans.append(xs_order[np.searchsorted(xs, a0):np.searchsorted(xs, b0, side="right")])
        if not spans:
            continue
        idx = np.unique(np.concatenate(spans))
        d = pos[idx] - centre[c]
        d -= np.round(d)
        r2 = np.einsum("ij,ij->i", d, d)
        t = 1.0 / (1.0 + r2 * (1.0 / a[c] ** 2))
        rho = (3.0 * per[c] / (4.0 * math.pi * a[c] ** 3 * umax[c])) * (t * t * np.sqrt(t))
        out[idx] += np.where(r2 < rmax[c] ** 2, rho, 0.0)
    return out


def batch_sizes(n_sets: int = 256, lo: float = 2e3, hi: float = 2e5, seed: int = 4) -> np.ndarray:
    """Set sizes log-uniform in [lo, hi] (the many-small-sets workload)."""
    rng = _rng(seed)
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_sets))).astype(np.int64)


def batch_sets(n_sets: int = 256, lo: float = 2e3, hi: float = 2e5, scale: float = 1.0):
    """The batched workload: set s is a clump/uniform mixture with seed 1000+s."""
    sizes = batch_sizes(n_sets, lo, hi)
    sizes = np.maximum(np.round(sizes * scale).astype(np.int64), 256)
    return [plummer_mixture(int(sz), 1000 + s) for s, sz in enumerate(sizes)]


def arrivals(n_req: int, rate_hz: float, lo: float = 1e4, hi: float = 2e6, seed: int = 5):
    """Poisson request stream: (arrival time [s], N) with N log-uniform in [lo, hi]."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    n = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_req))).astype(np.int64)
    return t, n
