"""Host checks of the seeded input generators used by the GPU tests: the
dense ball next to a top-cell face (the heavy-chunk and cell-order cases)
is reproducible, lies where its recipe says, and its first-guess h follows
the two number densities."""
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
