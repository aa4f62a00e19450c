"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to mathematics, physics or a number the
paper prints, so that a dropped term, a wrong sign or index or a transposed
operand anywhere in it fails at least one of them:

* kernel shape    -- equals the cubic B-spline from scipy's de Boor basis;
* normalisation   -- unit volume integral (quadrature) and the continuum
                     limit of lattice sums;
* derivatives     -- finite differences of the oracle's own W, rho, N_w;
* force           -- the pressure force is minus the gradient of the
                     thermal energy with h re-solved (grad-h Lagrangian);
* du/dt           -- the adiabatic rate (P/rho^2) drho/dt along the flow;
* viscosity       -- conservation, non-negative dissipation, linear in alpha,
                     and its magnitude, the sound speed and the signal
                     velocity on an isolated pair (plus a spectator), written
                     out with kernel derivatives by finite differences of the
                     B-spline and c^2 = dP/drho along the adiabat;
* neighbour sets  -- an independent scipy k-d tree, an independent
                     splitmix64, brute force vs the grid search;
* lattice         -- 56 neighbours inside h at N_w = 48 and zero force by
                     inversion symmetry;
* paper numbers   -- the in-range fractions printed in Sections II-B/II-C.
"""
import math

import numpy as np
import pytest
from scipy import integrate, interpolate, optimize
from scipy.spatial import cKDTree

import oracle
import sphinputs


# --------------------------------------------------------------------------
# kernel
# --------------------------------------------------------------------------
def test_kernel_is_cubic_bspline():
    # M4 kernel = cubic B-spline on knots -2..2 scaled to support 1, f(0)=1
    B = interpolate.BSpline.basis_element([-2, -1, 0, 1, 2], extrapolate=False)
    b0 = float(B(0.0))
    for q in np.linspace(0.0, 1.2, 241):
        ref = float(np.nan_to_num(B(2.0 * q))) / b0 if q < 1.0 else 0.0
        assert oracle.kernel_f(q) == pytest.approx(ref, abs=1e-14)
        dref = float(np.nan_to_num(B.derivative()(2.0 * q))) * 2.0 / b0 if q < 1.0 else 0.0
        assert oracle.kernel_df(q) == pytest.approx(dref, abs=1e-13)


@pytest.mark.parametrize("h", [0.37, 1.0, 3e-4])
def test_kernel_unit_volume(h):
    val, err = integrate.quad(lambda r: 4.0 * math.pi * r * r * oracle.W(r, h), 0.0, h,
                              points=[0.5 * h], epsabs=0, epsrel=1e-13)
    assert val == pytest.approx(1.0, rel=1e-11)


@pytest.mark.parametrize("r,h", [(0.1, 0.37), (0.3, 0.37), (0.2, 0.21), (0.7e-4, 2e-4)])
def test_kernel_derivatives_by_finite_difference(r, h):
    eh = 1e-6 * h
    fd_h = (oracle.W(r, h + eh) - oracle.W(r, h - eh)) / (2 * eh)
    assert oracle.dWdh(r, h) == pytest.approx(fd_h, rel=1e-6)
    er = 1e-6 * h
    fd_r = (oracle.W(r + er, h) - oracle.W(r - er, h)) / (2 * er)
    # grad_i W = k x_ij  =>  dW/dr = k r
    assert oracle.gradW_factor(r, h) * r == pytest.approx(fd_r, rel=1e-6)
    assert oracle.gradW_factor(r, h) < 0          # W decreases outward


def test_mix_matches_splitmix64_definition():
    M = (1 << 64) - 1

    def sm(x):
        z = (x + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    # first outputs of splitmix64 seeded with 0 are sm(0), sm(gamma), ...
    assert sm(0) == 0xE220A8397B1DCDAF
    for j in [0, 1, 2, 12345, 2 ** 40 + 7]:
        assert oracle.mix(j) == sm(j)


# --------------------------------------------------------------------------
# density: derivatives, normalisation, neighbour sets
# --------------------------------------------------------------------------
def test_density_h_derivatives_fd():
    ps = sphinputs.uniform(600, 11)
    h = np.full(ps.n, 0.2)
    t = np.arange(0, ps.n, 37)
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m, targets=t, brute=True)
    eps = 1e-6
    dp = oracle.density(ps.x, ps.y, ps.z, h * (1 + eps), ps.m, targets=t, brute=True)
    dm = oracle.density(ps.x, ps.y, ps.z, h * (1 - eps), ps.m, targets=t, brute=True)
    fd_rho = (dp["rho"] - dm["rho"])[t] / (2 * eps * h[t])
    fd_nw = (dp["nw"] - dm["nw"])[t] / (2 * eps * h[t])
    assert np.allclose(d["drho_dh"][t], fd_rho, rtol=1e-5, atol=1e-9 * np.abs(fd_rho).max())
    assert np.allclose(d["dnw_dh"][t], fd_nw, rtol=1e-5, atol=1e-9 * np.abs(fd_nw).max())


def test_nw_is_kernel_volume_times_number_density():
    # equal masses: N_w = (4 pi / 3) h^3 rho / m, from two separately coded sums
    ps = sphinputs.plummer_mixture(3000, 3)
    d = oracle.density(ps.x, ps.y, ps.z, ps.h0, ps.m)
    lhs = d["nw"]
    rhs = 4.0 * math.pi / 3.0 * ps.h0 ** 3 * d["rho"] / ps.m
    assert np.allclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("hs,tol", [(3.0, 3e-3), (4.0, 1e-3)])
def test_lattice_continuum_limit(hs, tol):
    # a lattice sum of a unit-volume kernel tends to the number density
    n_side = 16
    ps = sphinputs.lattice(n_side, 0.0, 0)
    dlt = 1.0 / n_side
    h = np.full(ps.n, hs * dlt)
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m, targets=[0, 100, 2000])
    val = d["rho"][[0, 100, 2000]] * dlt ** 3 / ps.m[0]
    assert np.all(np.abs(val - 1.0) < tol)
    assert np.ptp(val) < 1e-12


def test_lattice_solved_h_pins():
    # Perfect lattice, N_w = 48: 56 neighbours (shells r^2 <= 5 spacings^2),
    # zero force by inversion symmetry, and the root agrees with an
    # independent shell-sum root found by brentq on scipy's B-spline.
    n_side = 16
    dlt = 1.0 / n_side
    ps = sphinputs.lattice(n_side, 0.0, 0)
    h, it = oracle.solve_h(ps.x, ps.y, ps.z, ps.m, ps.h0, tol=1e-12)
    assert np.ptp(h) < 1e-12
    hs = h[0] / dlt
    assert math.sqrt(5) < hs < math.sqrt(6)
    B = interpolate.BSpline.basis_element([-2, -1, 0, 1, 2], extrapolate=False)
    b0 = float(B(0.0))
    k = np.arange(-4, 5)
    I, J, K = np.meshgrid(k, k, k, indexing="ij")
    r = np.sqrt(I ** 2 + J ** 2 + K ** 2).ravel()

    def nw(s):
        q = r / s
        vals = np.nan_to_num(B(2.0 * q[q < 1])) / b0
        return 4.0 * math.pi / 3.0 * s ** 3 * (8.0 / math.pi / s ** 3) * vals.sum() - 48.0

    root = optimize.brentq(nw, 2.0, 2.4, xtol=1e-15)
    assert hs == pytest.approx(root, rel=1e-10)
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m)
    assert np.all(d["nngb"] == 56)
    assert np.allclose(d["nw"], 48.0, atol=1e-9)
    f = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, d["rho"], d["drho_dh"])
    amag = np.sqrt(f["ax"] ** 2 + f["ay"] ** 2 + f["az"] ** 2)
    assert np.all(amag <= 1e-12 * f["S"])
    assert np.all(f["nforce"] == 56)


def _ckdtree_sets(ps, h):
    pos = np.mod(ps.pos(), 1.0)
    tree = cKDTree(pos, boxsize=1.0)
    hmax = h.max()
    pairs = tree.query_pairs(hmax, output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    d = pos[i] - pos[j]
    d -= np.round(d)
    r = np.sqrt((d * d).sum(1))
    return i, j, r


def _sm(x):
    M = (1 << 64) - 1
    z = (int(x) + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


@pytest.mark.parametrize("recipe", ["uniform", "plummer"])
def test_neighbour_sets_against_kdtree(recipe):
    ps = sphinputs.uniform(3000, 5) if recipe == "uniform" else sphinputs.plummer_mixture(4000, 6)
    h = ps.h0
    i, j, r = _ckdtree_sets(ps, h)
    n = ps.n
    dens = np.zeros(n, dtype=np.int64)
    forc = np.zeros(n, dtype=np.int64)
    hashd = [0] * n
    M = (1 << 64) - 1
    inn_i = r < h[i]
    inn_j = r < h[j]
    np.add.at(dens, i[inn_i], 1)
    np.add.at(dens, j[inn_j], 1)
    for a, b in zip(i[inn_i], j[inn_i]):
        hashd[a] = (hashd[a] + _sm(b)) & M
    for a, b in zip(i[inn_j], j[inn_j]):
        hashd[b] = (hashd[b] + _sm(a)) & M
    fm = r < np.maximum(h[i], h[j])
    np.add.at(forc, i[fm], 1)
    np.add.at(forc, j[fm], 1)
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m)
    assert np.array_equal(d["nngb"], dens)
    assert [int(v) for v in d["hash"]] == hashd
    z = np.zeros(n)
    f = oracle.force(ps.x, ps.y, ps.z, h, ps.m, z, z, z, ps.u, d["rho"], d["drho_dh"])
    assert np.array_equal(f["nforce"], forc)


@pytest.mark.parametrize("recipe", ["uniform", "plummer"])
def test_grid_equals_brute_force(recipe):
    ps = (sphinputs.uniform(2500, 7, velocity=True) if recipe == "uniform"
          else sphinputs.plummer_mixture(3000, 8, velocity=True))
    h = ps.h0
    assert h.max() / h.min() > (1.5 if recipe == "uniform" else 30) or recipe == "uniform"
    dg = oracle.density(ps.x, ps.y, ps.z, h, ps.m)
    db = oracle.density(ps.x, ps.y, ps.z, h, ps.m, brute=True)
    assert np.array_equal(dg["nngb"], db["nngb"]) and np.array_equal(dg["hash"], db["hash"])
    for k in ("rho", "drho_dh", "nw", "dnw_dh"):
        assert np.allclose(dg[k], db[k], rtol=1e-12, atol=0)
    fg = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, dg["rho"], dg["drho_dh"])
    fb = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, dg["rho"], dg["drho_dh"],
                      brute=True)
    assert np.array_equal(fg["nforce"], fb["nforce"]) and np.array_equal(fg["hash"], fb["hash"])
    for k in ("ax", "ay", "az", "dudt", "S", "vsig"):
        assert np.allclose(fg[k], fb[k], rtol=1e-10, atol=1e-12 * np.abs(fb["S"]).max())


def test_periodic_translation_invariance():
    ps = sphinputs.uniform(2000, 9)
    h = ps.h0
    d0 = oracle.density(ps.x, ps.y, ps.z, h, ps.m)
    sh = np.array([0.25, 0.5 + 2 ** -24 * 3, 0.875])
    x = np.mod(ps.x + sh[0], 1.0)
    y = np.mod(ps.y + sh[1], 1.0)
    z = np.mod(ps.z + sh[2], 1.0)
    d1 = oracle.density(x, y, z, h, ps.m)
    assert np.array_equal(d0["nngb"], d1["nngb"]) and np.array_equal(d0["hash"], d1["hash"])
    assert np.allclose(d0["rho"], d1["rho"], rtol=1e-13)


# --------------------------------------------------------------------------
# force: Lagrangian derivation, adiabatic du/dt, conservation, viscosity
# --------------------------------------------------------------------------
def _resolve(x, y, z, m, h0):
    h, _ = oracle.solve_h(x, y, z, m, h0, brute=True, tol=1e-13, max_iter=200)
    return h


def test_pressure_force_is_energy_gradient():
    # With h re-solved to N_w = 48 (equal masses: rho h^3 fixed) and
    # entropies K_j fixed, m_i a_i = -dU/dx_i with U = sum_j m_j u_j(rho_j).
    rng = np.random.default_rng(3)
    n = 300
    pos = rng.random((n, 3))
    m = np.full(n, 1.0 / n)
    u0 = 1.0 + rng.random(n)
    g = oracle.GAMMA
    x, y, z = pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy()
    h = _resolve(x, y, z, m, np.full(n, 0.33))
    d = oracle.density(x, y, z, h, m, brute=True)
    K = (g - 1.0) * u0 / d["rho"] ** (g - 1.0)
    zero = np.zeros(n)
    f = oracle.force(x, y, z, h, m, zero, zero, zero, u0, d["rho"], d["drho_dh"], alpha=0.0,
                     brute=True)

    def U(xx, yy, zz):
        hh = _resolve(xx, yy, zz, m, h)
        rr = oracle.density(xx, yy, zz, hh, m, brute=True)["rho"]
        return float(np.sum(m * K * rr ** (g - 1.0) / (g - 1.0)))

    delta = 1e-6
    for i in [0, 17, 123]:
        grad = []
        for comp in range(3):
            p = [x.copy(), y.copy(), z.copy()]
            q = [x.copy(), y.copy(), z.copy()]
            p[comp][i] += delta
            q[comp][i] -= delta
            grad.append((U(*p) - U(*q)) / (2 * delta))
        ma = m[i] * np.array([f["ax"][i], f["ay"][i], f["az"][i]])
        scale = m[i] * f["S"][i]
        assert np.allclose(ma, -np.array(grad), rtol=1e-5, atol=1e-6 * scale)


def test_dudt_is_adiabatic_rate():
    rng = np.random.default_rng(4)
    n = 300
    pos = rng.random((n, 3))
    v = rng.uniform(-1, 1, (n, 3))
    m = np.full(n, 1.0 / n)
    u = 1.0 + rng.random(n)
    x, y, z = pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy()
    h = _resolve(x, y, z, m, np.full(n, 0.33))
    d = oracle.density(x, y, z, h, m, brute=True)
    f = oracle.force(x, y, z, h, m, v[:, 0], v[:, 1], v[:, 2], u, d["rho"], d["drho_dh"],
                     alpha=0.0, brute=True)
    dt = 1e-6
    rp = []
    for s in (+1, -1):
        xx, yy, zz = x + s * dt * v[:, 0], y + s * dt * v[:, 1], z + s * dt * v[:, 2]
        hh = _resolve(xx, yy, zz, m, h)
        rp.append(oracle.density(xx, yy, zz, hh, m, brute=True)["rho"])
    drho_dt = (rp[0] - rp[1]) / (2 * dt)
    P = (oracle.GAMMA - 1.0) * d["rho"] * u
    ref = P / d["rho"] ** 2 * drho_dt
    assert np.allclose(f["dudt"], ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())


@pytest.mark.parametrize("alpha", [0.0, 2.0])
def test_conservation(alpha):
    ps = sphinputs.plummer_mixture(4000, 12, velocity=True)
    h, _ = oracle.solve_h(ps.x, ps.y, ps.z, ps.m, ps.h0)
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m)
    f = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, d["rho"], d["drho_dh"],
                     alpha=alpha)
    s = oracle.sums(ps.m, ps.vx, ps.vy, ps.vz, f["ax"], f["ay"], f["az"], f["dudt"], f["S"])
    assert np.all(np.abs(s["M"]) <= 1e-12 * s["scale"])
    assert abs(s["E"]) <= 1e-12 * s["scale"]
    # the force pair relation is symmetric: each unordered pair is counted twice
    assert f["nforce"].sum() % 2 == 0


def test_viscosity_dissipates_and_is_linear_in_alpha():
    ps = sphinputs.uniform(2000, 13, velocity=True)
    h, _ = oracle.solve_h(ps.x, ps.y, ps.z, ps.m, ps.h0)
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m)
    out = {}
    for a in (0.0, 1.0, 2.0):
        out[a] = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, d["rho"],
                              d["drho_dh"], alpha=a)
    heat = np.sum(ps.m * (out[2.0]["dudt"] - out[0.0]["dudt"]))
    assert heat > 0
    for k in ("ax", "ay", "az", "dudt"):
        lin = out[2.0][k] - out[0.0][k] - 2.0 * (out[1.0][k] - out[0.0][k])
        assert np.allclose(lin, 0.0, atol=1e-11 * np.abs(out[2.0]["S"]).max())
    # at rest the viscosity vanishes identically
    z = np.zeros(ps.n)
    f0 = oracle.force(ps.x, ps.y, ps.z, h, ps.m, z, z, z, ps.u, d["rho"], d["drho_dh"], alpha=0.0)
    f2 = oracle.force(ps.x, ps.y, ps.z, h, ps.m, z, z, z, ps.u, d["rho"], d["drho_dh"], alpha=2.0)
    assert np.array_equal(f0["ax"], f2["ax"]) and np.array_equal(f0["dudt"], f2["dudt"])


def test_two_particles_newton_third_law():
    x = np.array([0.40, 0.40 + 0.05])
    y = np.array([0.5, 0.5])
    z = np.array([0.5, 0.5])
    h = np.array([0.08, 0.12])
    m = np.array([1.0, 2.0])
    u = np.array([1.0, 3.0])
    d = oracle.density(x, y, z, h, m, brute=True)
    zero = np.zeros(2)
    f = oracle.force(x, y, z, h, m, zero, zero, zero, u, d["rho"], d["drho_dh"], brute=True)
    assert f["ax"][0] < 0 < f["ax"][1]                      # pressure pushes apart
    assert m[0] * f["ax"][0] == pytest.approx(-m[1] * f["ax"][1], rel=1e-14)
    assert f["ay"][0] == 0 and f["az"][1] == 0
    # only j = 1 is inside h_0 (0.05 < 0.08): one density neighbour each
    assert list(d["nngb"]) == [1, 1]
    # across the periodic face the same pair gives the same result
    x2 = np.array([0.99, 0.99 + 0.05 - 1.0])
    d2 = oracle.density(x2, y, z, h, m, brute=True)
    f2 = oracle.force(x2, y, z, h, m, zero, zero, zero, u, d2["rho"], d2["drho_dh"], brute=True)
    assert f2["ax"][0] == pytest.approx(f["ax"][0], rel=1e-12)


def test_single_particle():
    x = np.array([0.3]); y = np.array([0.6]); z = np.array([0.9])
    d = oracle.density(x, y, z, [0.2], [2.0])
    assert d["nngb"][0] == 0 and d["hash"][0] == 0
    # N_w of an isolated particle is the kernel volume times W(0): its own term
    assert d["nw"][0] == pytest.approx(4.0 * math.pi / 3.0 * 0.2 ** 3 * oracle.W(0.0, 0.2))
    f = oracle.force(x, y, z, [0.2], [2.0], [0.0], [0.0], [0.0], [1.0], d["rho"], d["drho_dh"])
    assert f["ax"][0] == 0 and f["nforce"][0] == 0


# --------------------------------------------------------------------------
# the paper's printed statistics
# --------------------------------------------------------------------------
def test_best_case_in_range_fraction(paper):
    # Section II-B: with h equal to the cell edge, ~16% of the particles in a
    # particle's own and neighbouring cells are within range.
    n = 20000
    ps = sphinputs.uniform(n, 21)
    G = 8
    h = np.full(n, 1.0 / G)
    d = oracle.density(ps.x, ps.y, ps.z, h, ps.m)
    frac = d["nngb"].mean() / (27.0 * n / G ** 3)
    assert abs(frac - paper["best_case_in_range"]) < 0.01


def test_face_pair_in_range_fraction(paper):
    # Section II-C: 33.5% of the naive cross pairs of two face-sharing cells
    # (edge h, uniform particles) are in range.
    rng = np.random.default_rng(22)
    n = 3000
    h = 0.1
    a = rng.random((n, 3)) * h + 0.3
    b = rng.random((n, 3)) * h + 0.3
    b[:, 0] += h
    allp = np.concatenate([a, b])
    hh = np.full(2 * n, h)
    m = np.ones(2 * n)
    both = oracle.density(allp[:, 0], allp[:, 1], allp[:, 2], hh, m)["nngb"][:n].sum()
    only = oracle.density(a[:, 0], a[:, 1], a[:, 2], hh[:n], m[:n])["nngb"].sum()
    frac = (both - only) / float(n * n)
    assert abs(frac - paper["face_in_range"]) < 0.004


# --------------------------------------------------------------------------
# viscosity, sound speed and signal velocity: two particles in closed form
# --------------------------------------------------------------------------
_BS = interpolate.BSpline.basis_element([-2, -1, 0, 1, 2], extrapolate=False)
_BS0 = float(_BS(0.0))


def _W_bspline(r, h):
    """Cubic-spline kernel from scipy's de Boor basis (support radius h, unit
    volume: the normalisation 8/(pi h^3) of f(0) = 1 is the quadrature pin
    above), independent of the oracle's polynomial pieces."""
    q = r / h
    f = float(np.nan_to_num(_BS(2.0 * q))) / _BS0 if q < 1.0 else 0.0
    return 8.0 / (math.pi * h ** 3) * f


def _dWdr(r, h):
    e = 1e-5 * h
    return (_W_bspline(r + e, h) - _W_bspline(r - e, h)) / (2 * e)


def _sound_speed(rho, u, gamma):
    """Adiabatic sound speed sqrt(dP/drho at constant entropy) of the ideal
    gas P = (gamma-1) rho u, by a central difference along the adiabat
    u(rho') = u (rho'/rho)^(gamma-1)."""
    def P(r):
        return (gamma - 1.0) * r * u * (r / rho) ** (gamma - 1.0)
    e = 1e-5 * rho
    return math.sqrt((P(rho + e) - P(rho - e)) / (2 * e))


def _two_particle_reference(r, h, m, u, v, gamma, alpha, spec, mutate=None):
    """Density and force of particle 0 of a pair on the x axis (particle 1 at
    +r), written out from the definitions: density sums over j within h_i
    (self included), grad-h factor from a finite difference of rho(h),
    ideal-gas pressure, the signal-velocity viscosity of the chosen reading,
    and the force/energy sums over j within max(h_i, h_j).  A spectator
    particle 2 at rest sits a distance s from particle 0 along y: it adds to
    the densities (so that no particle is alone in its own h, where the
    grad-h factor is singular) but not to the x force or du/dt of particle 0
    (its pair with 0 is perpendicular to x and to the velocities).
    mutate names a plausible mistake to apply (the test shows each one moves
    the result far outside the tolerance)."""
    s, m2, u2 = spec
    d = [[0.0, r, s], [r, 0.0, math.hypot(r, s)]]   # distances of 0 and 1 to 0, 1, 2
    mm = [m[0], m[1], m2]

    def rho_of(i, hh):
        return sum(mm[j] * _W_bspline(d[i][j], hh) for j in range(3) if d[i][j] < hh or j == i)

    rho = [rho_of(0, h[0]), rho_of(1, h[1])]
    drho = [(rho_of(i, h[i] * (1 + 1e-6)) - rho_of(i, h[i] * (1 - 1e-6))) / (2e-6 * h[i]) for i in (0, 1)]
    fgr = [1.0 / (1.0 + h[i] / (3.0 * rho[i]) * drho[i]) for i in (0, 1)]
    Pr = [(gamma - 1.0) * rho[i] * u[i] for i in (0, 1)]
    if mutate == "c_sqrt_gamma_u":
        c = [math.sqrt(gamma * uu) for uu in (u[0], u[1], u2)]
    else:
        c = [_sound_speed(rho[i], u[i], gamma) for i in (0, 1)] + [_sound_speed(1.0, u2, gamma)]
    A = [fgr[i] * Pr[i] / rho[i] ** 2 for i in (0, 1)]
    out = {"rho": rho[0], "c": c[0], "A": A[0]}
    # x_01 = x_0 - x_1 = -r along x; grad_0 W(r, h) = dW/dr * x_01 / r
    xij = -r
    vij = v[0] - v[1]
    w = vij * xij / r
    Gi = (_dWdr(r, h[0]) if r < h[0] else 0.0) * xij / r
    Gj = (_dWdr(r, h[1]) if r < h[1] else 0.0) * xij / r
    Gbar = 0.5 * (Gi + Gj)
    a_eff = 0.25 * alpha if mutate == "alpha_half" else 0.5 * alpha
    rhobar = (rho[0] + rho[1]) if mutate == "rho_sum" else 0.5 * (rho[0] + rho[1])
    beta = 0.0 if mutate == "no_minus_3w" else 3.0
    Pi = -a_eff * (c[0] + c[1] - beta * w) * w / rhobar if w < 0 else 0.0
    out["ax"] = -m[1] * (A[0] * Gi + A[1] * Gj + Pi * Gbar)
    out["dudt"] = m[1] * (A[0] * vij * Gi + 0.5 * Pi * vij * Gbar)
    # the spectator is at rest and met perpendicular to the flow: w = 0
    out["vsig"] = max(c[0] + c[1] - beta * min(w, 0.0), c[0] + c[2])
    return out


_PAIR_CASES = {
    # approaching, both within each other's h
    "approaching": dict(x0=0.40, r=0.05, h=(0.08, 0.12), v=(0.7, -0.4)),
    # receding: no viscosity, v_sig is the sum of the sound speeds
    "receding": dict(x0=0.40, r=0.05, h=(0.08, 0.12), v=(-0.3, 0.5)),
    # r between the two h: only particle 1 sees particle 0 in its density
    "one_sided": dict(x0=0.30, r=0.10, h=(0.08, 0.12), v=(0.9, -0.2)),
    # the same approaching pair across the periodic face x = 0 = 1
    "periodic": dict(x0=0.98, r=0.05, h=(0.08, 0.12), v=(0.7, -0.4)),
}


@pytest.mark.parametrize("name", list(_PAIR_CASES))
def test_two_particle_viscosity_closed_form(name):
    cs = _PAIR_CASES[name]
    r, h, v = cs["r"], cs["h"], cs["v"]
    m, u, gamma, alpha = (1.0, 2.0), (1.0, 3.0), 5.0 / 3.0, 2.0
    spec = (0.5 * h[0], 1.5, 0.2)
    x = np.array([cs["x0"], math.fmod(cs["x0"] + r, 1.0), cs["x0"]])
    y = np.array([0.5, 0.5, 0.5 + spec[0]])
    z = np.array([0.5, 0.5, 0.5])
    hh = np.array([h[0], h[1], 0.05])
    mm = np.array([m[0], m[1], spec[1]])
    uu = np.array([u[0], u[1], spec[2]])
    d = oracle.density(x, y, z, hh, mm, brute=True)
    g = oracle.ghost(hh, d["rho"], d["drho_dh"], uu, gamma)
    vx = np.array([v[0], v[1], 0.0])
    zero = np.zeros(3)
    f = oracle.force(x, y, z, hh, mm, vx, zero, zero, uu, d["rho"], d["drho_dh"],
                     gamma=gamma, alpha=alpha, brute=True)
    ref = _two_particle_reference(r, h, m, u, v, gamma, alpha, spec)
    # finite differences of the kernel and of the adiabat carry ~1e-9
    assert d["rho"][0] == pytest.approx(ref["rho"], rel=1e-9)
    assert g["c"][0] == pytest.approx(ref["c"], rel=1e-8)
    assert g["A"][0] == pytest.approx(ref["A"], rel=1e-7)
    assert f["ax"][0] == pytest.approx(ref["ax"], rel=1e-6)
    assert f["dudt"][0] == pytest.approx(ref["dudt"], rel=1e-6, abs=1e-12)
    assert f["vsig"][0] == pytest.approx(ref["vsig"], rel=1e-8)
    assert f["az"][0] == 0.0
    # each plausible misreading moves some result far outside those bars
    # (the receding pair has no viscosity, so only the sound speed shows)
    mutations = ["c_sqrt_gamma_u"] if name == "receding" else \
        ["alpha_half", "rho_sum", "no_minus_3w", "c_sqrt_gamma_u"]
    for mu in mutations:
        bad = _two_particle_reference(r, h, m, u, v, gamma, alpha, spec, mutate=mu)
        moved = max(abs(bad[k] / ref[k] - 1.0) for k in ("ax", "dudt", "vsig", "c") if ref[k] != 0.0)
        assert moved > 1e-3, mu
