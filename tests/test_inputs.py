"""Host checks of the seeded input generators used by the GPU tests and
the benchmark: the dense ball next to a top-cell face (the heavy-chunk and
cell-order cases) and the Plummer-clump mixture (the multi-resolution
workload) are reproducible, lie where their recipes say, and their
first-guess h follows their number densities."""
import numpy as np

import sphinputs


def test_clump_by_face_recipe():
    a = sphinputs.clump_by_face(2000, 6000, 5)
    b = sphinputs.clump_by_face(2000, 6000, 5)
    assert a.n == 8000
    for k in ("x", "y", "z", "h0", "m"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    ball = np.stack([a.x[2000:], a.y[2000:], a.z[2000:]], axis=1)
    r = np.linalg.norm(ball - np.array([0.535, 0.375, 0.375]), axis=1)
    assert r.max() <= 0.03 + 1e-6
    # the ball lies wholly past the plane x = 1/2 (a top-cell face)
    assert ball[:, 0].min() > 0.5
    bg = np.stack([a.x[:2000], a.y[:2000], a.z[:2000]], axis=1)
    assert bg.min() >= 0.0 and bg.max() < 1.0
    # first-guess h: the background's from its density, the ball's smaller
    # by the cube root of the density ratio
    h_bg = sphinputs.h_for_density(2000.0)
    assert np.allclose(a.h0[:2000], np.float32(h_bg), rtol=1e-6)
    ratio = (2000.0 + 6000 / (4.0 / 3.0 * np.pi * 0.03 ** 3)) / 2000.0
    assert np.allclose(a.h0[2000:], np.float32(h_bg / np.cbrt(ratio)), rtol=1e-6)
    # distinct positions
    assert len(np.unique(np.stack([a.x, a.y, a.z], axis=1), axis=0)) == a.n


def test_plummer_mixture_recipe():
    """One clump plus 20% background: reproducible; the clump's radii, drawn
    by inverting its enclosed-mass fraction, follow the analytic number
    density that gives the first-guess h (integrated over radial shells,
    within Poisson noise), and that density integrates to the clump's
    particle count."""
    from scipy.integrate import simpson

    n = 40000
    a = sphinputs.plummer_mixture(n, 11, n_clumps=1)
    b = sphinputs.plummer_mixture(n, 11, n_clumps=1)
    for k in ("x", "y", "z", "h0"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    n_bg, n_c = 8000, 32000
    ac = float(a.meta["a"][0])
    centre = np.array(a.meta["centre"][0])
    rmax = min(20.0 * ac, 0.45)
    pos = np.stack([a.x, a.y, a.z], axis=1)
    assert pos.min() >= 0.0 and pos.max() < 1.0
    d = pos[n_bg:] - centre
    d -= np.round(d)
    r = np.linalg.norm(d, axis=1)
    assert r.max() <= rmax + 1e-6

    def rho(rr):
        pts = np.mod(centre + rr[:, None] * np.array([1.0, 0.0, 0.0]), 1.0)
        return sphinputs.plummer_number_density(pts, n_bg, np.array([n_c]), np.array([ac]), np.array([rmax]),
                                                centre[None, :]) - n_bg

    def count(r0, r1):
        rr = np.geomspace(max(r0, 1e-9 * rmax), r1, 4001)
        return simpson(4.0 * np.pi * rr ** 2 * rho(rr), x=rr)

    assert abs(count(0.0, rmax * (1 - 1e-12)) - n_c) < 1e-3 * n_c
    edges = rmax * np.array([0.0, 0.02, 0.05, 0.1, 0.2, 0.4, 0.7, 1.0 - 1e-12])
    for r0, r1 in zip(edges[:-1], edges[1:]):
        exp = count(r0, r1)
        got = np.count_nonzero((r >= r0) & (r < r1))
        assert abs(got - exp) <= 5.0 * np.sqrt(exp) + 5.0, (r0, r1, got, exp)
    # the first guess: h for the analytic density at each particle
    dens = sphinputs.plummer_number_density(pos, n_bg, np.array([n_c]), np.array([ac]), np.array([rmax]),
                                            centre[None, :])
    assert np.array_equal(a.h0, np.float32(sphinputs.h_for_density(dens)).astype(np.float64))


def test_jittered_lattice_recipe():
    """The headline workload's generator (at 20^3): every particle within
    the jitter of its own lattice point (periodic), positions on the 2^-24
    grid and distinct, equal masses summing to one, and the first-guess h
    that of the mean number density."""
    ns, jit = 20, 0.1
    a = sphinputs.lattice(ns, jit, 2)
    assert a.n == ns ** 3
    d = 1.0 / ns
    g = (np.arange(ns) + 0.5) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    base = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pos = np.stack([a.x, a.y, a.z], axis=1)
    off = pos - base
    off -= np.round(off)
    assert np.abs(off).max() <= jit * d + 2.0 ** -24
    assert np.array_equal(pos * 2.0 ** 24, np.floor(pos * 2.0 ** 24))
    assert len(np.unique(pos, axis=0)) == a.n
    assert np.all(a.m == a.m[0]) and abs(a.m.sum() - 1.0) < 1e-6
    assert np.all(a.h0 == np.float32(sphinputs.h_for_density(float(a.n))))
