"""GPU tests of the cell-order reads: a partner whose swept prefix is long
is read in cell order, and the 64-particle blocks of it that lie beyond a
chunk's reach are passed over without being loaded.

* passing over blocks is bitwise neutral: every output equals the one of
  reading every particle of such a partner (SPH_FLAG_NO_BLOCK_SKIP), at a
  fixed h and through the Newton solve of h;
* against sweeping every partner through its sorted lists
  (SPH_FLAG_SORTED_ONLY) the pair sets and counts are bit-exact and the sums
  agree to rounding, with fewer records loaded (sph_last_reads: the path
  was taken);
* the oracle, element by element, on sets where the path is taken.
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

from _checks import check_density, check_force, full_check, run_fixed  # noqa: E402


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


def _case(name):
    """(particles, h, build parameters): a dense ball just past a top-cell
    face (background leaves on the other side sweep the whole ball) and a
    uniform set on two top cells per side with no refinement (top cells of
    ~5000 particles)."""
    if name == "clumpy":
        ps = sphinputs.clump_by_face(8000, 30000, 77, velocity=True)
        ps, h = I.fixed_h_case(ps)
        return ps, h, {}
    ps = sphinputs.uniform(40000, 8, velocity=True)
    h = I.f32(np.full(ps.n, sphinputs.h_for_density(float(ps.n))))
    ps = I.redraw_ties_uniform(ps, h, seed=108)
    return ps, h, {"top_grid": 2, "n_split": 1 << 30}


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("name", ["clumpy", "uniform_two_top_cells"])
def test_block_skip_is_bitwise_neutral(sph, ctx, name):
    ps, h, kw = _case(name)
    (g,), _ = run_fixed(sph, ctx, [ps], [h], **kw)
    r_skip = ctx.reads()
    (g2,), _ = run_fixed(sph, ctx, [ps], [h], flags=sph.SPH_FLAG_NO_BLOCK_SKIP, **kw)
    r_all = ctx.reads()
    _same(g[0], g2[0])
    _same(g[1], g2[1])
    # blocks were passed over in both stages (where the dense ball is read
    # in cell order)
    print(f"records loaded (density, force): {r_skip} passing over blocks, {r_all} reading all")
    assert r_skip[0] <= r_all[0] and r_skip[1] <= r_all[1]
    if name == "clumpy":
        assert r_skip[0] < r_all[0] and r_skip[1] < r_all[1]


@pytest.mark.parametrize("name", ["clumpy", "uniform_two_top_cells"])
def test_cell_order_matches_sorted_sweeps(sph, ctx, name):
    ps, h, kw = _case(name)
    (g,), tg = run_fixed(sph, ctx, [ps], [h], **kw)
    r_cell = ctx.reads()
    (s,), ts = run_fixed(sph, ctx, [ps], [h], flags=sph.SPH_FLAG_SORTED_ONLY, **kw)
    r_sorted = ctx.reads()
    for k in ("nngb", "hash", "h"):
        assert np.array_equal(g[0][k], s[0][k]), k
    for k in ("nforce", "hash"):
        assert np.array_equal(g[1][k], s[1][k]), k
    assert np.allclose(g[0]["rho"], s[0]["rho"], rtol=2e-6, atol=0)
    scale = np.maximum(g[1]["S"], 1e-30)
    for k in ("ax", "ay", "az", "dudt"):
        assert np.max(np.abs(g[1][k] - s[1][k]) / scale) < 1e-5, k
    # clumpy: the cell-order reads were used where the ball is, and loaded
    # fewer records.  Two top cells per side: the top cells (~5000
    # particles) have no sorted lists unless all lists are asked for, and
    # are read in cell order (more records loaded than the axial slabs, for
    # no sort)
    print(f"records loaded (density, force): {r_cell} with cell-order reads, {r_sorted} sorted sweeps only")
    if name == "clumpy":
        assert r_cell[0] < r_sorted[0] and r_cell[1] < r_sorted[1]
    else:
        assert tg.stats()["sorted_entries"] == 0 < ts.stats()["sorted_entries"]


@pytest.mark.parametrize("name", ["clumpy", "uniform_two_top_cells"])
def test_cell_order_against_oracle(sph, ctx, name):
    ps, h, kw = _case(name)
    if kw:
        (g,), _ = run_fixed(sph, ctx, [ps], [h], **kw)
        rd, rf = I.oracle_reference(ps, h)
        check_density(ps, h, g[0], rd)
        check_force(ps, g[1], rf)
    else:
        full_check(sph, ctx, ps, h)


def test_block_skip_neutral_through_the_solve(sph, ctx):
    # the Newton passes run on the unconverged particles only, whose
    # bounding boxes per chunk are smaller: still bitwise the same h
    ps = sphinputs.clump_by_face(8000, 30000, 78, velocity=True)
    batch = sph.batch_from_sets([ps])
    res = []
    for flags in (0, sph.SPH_FLAG_NO_BLOCK_SKIP):
        prm = sph.params(flags=flags)
        tree = sph.Tree(ctx)
        d = sph.DensityOut(ps.n, "cuda")
        st, nu, it = sph.solve_with_rebuild(tree, batch, prm, d)
        assert st == sph.SPH_OK and nu == 0
        f = sph.ForceOut(ps.n, 1, "cuda")
        tree.force(f)
        torch.cuda.synchronize()
        res.append((d.h.cpu().numpy(), d.rho.cpu().numpy(), f.ax.cpu().numpy(), f.dudt.cpu().numpy(), it))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
