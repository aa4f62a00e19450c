"""GPU parity on inputs that are not on the 2^-24 grid.

The other parity cases snap positions to k 2^-24, where every offset inside
a top cell is exact in FP32.  Here positions keep all their FP64 bits: a
clumpy set whose h spans more than 2.5 decades (smallest h under 1/300 of
the top cell edge), a jittered lattice after one FP64 drift step with its
velocities (the state a time step leaves), and a fixed h three times the
solved one (~1300 neighbours per particle, past the length where a plain
FP32 density sum could still be bounded by the tolerance).  All use the
fixed-h protocol (h from the oracle's solve, raised until no pair lies
within 1e-6 of a cutoff) and the full bar: pair sets and counts exact,
density 1e-5, force 1e-4 of S_i.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import _inputs as I  # noqa: E402

import sphinputs  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from _checks import full_check  # noqa: E402


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1309_3783_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(sph):
    return sph.Context(0)


def _report(name, ps, h, g, rd, rf):
    e_rho = float((np.abs(g[0]["rho"] - rd["rho"]) / rd["rho"]).max())
    S = np.maximum(rf["S"], 1e-300)
    e_a = float(max((np.abs(g[1][k] - rf[k]) / S).max() for k in ("ax", "ay", "az")))
    print(f"\n[offgrid] {name}: n {ps.n} h {h.min():.3g}..{h.max():.3g} mean nngb {g[0]['nngb'].mean():.1f} "
          f"rho rel {e_rho:.2e} a/S {e_a:.2e}", flush=True)


def test_offgrid_clumpy_wide_h_range(sph, ctx):
    ps = sphinputs.plummer_mixture(40000, 41, n_clumps=8, snap=False, velocity=True)
    assert not np.all(ps.x * 2.0 ** 24 == np.floor(ps.x * 2.0 ** 24))
    ps, h = I.fixed_h_case(ps)
    assert h.max() / h.min() > 10 ** 2.5
    g, rd, rf, tree = full_check(sph, ctx, ps, h)
    st = tree.stats()
    assert h.min() * st["top_grid"] < 1.0 / 300.0, st      # h_min / L0
    assert st["levels"] >= 4, st
    _report("clumpy", ps, h, g, rd, rf)


def test_offgrid_drifted_lattice(sph, ctx):
    ps = sphinputs.lattice(24, 0.1, 2, velocity=True)
    # one drift step in FP64, as sph_drift makes it: x += dt v, wrapped (a
    # step that is not a power of two: dt v then has bits far below 2^-24)
    dt = 0.1234567
    ps.x = np.mod(ps.x + dt * ps.vx, 1.0)
    ps.y = np.mod(ps.y + dt * ps.vy, 1.0)
    ps.z = np.mod(ps.z + dt * ps.vz, 1.0)
    assert np.mean(ps.x * 2.0 ** 24 == np.floor(ps.x * 2.0 ** 24)) < 0.01
    ps, h = I.fixed_h_case(ps)
    g, rd, rf, _ = full_check(sph, ctx, ps, h)
    _report("drifted lattice", ps, h, g, rd, rf)


def test_offgrid_many_neighbours(sph, ctx):
    ps = sphinputs.lattice(24, 0.1, 3, velocity=True, snap=False)
    h3 = 3.0 * I.solved_h(ps)
    ps, h = I.fixed_h_case(ps, h3)
    g, rd, rf, tree = full_check(sph, ctx, ps, h)
    assert g[0]["nngb"].mean() > 1000
    _report("3x h", ps, h, g, rd, rf)
