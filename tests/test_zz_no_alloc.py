"""The entry point that allocates nothing: sph_build_cells_static builds the
tree in the library's static scratch (a file-scope device array), so neither
it nor the calls that follow on the tree allocate device memory.  Checked
through the C-ABI against sph_build_cells on the same inputs, on two calls
in a row (the second with a smaller set): the outputs must be the same bit
for bit (same kernels, same data; only the memory differs).
"""
import ctypes as C
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

import sphinputs  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1309_3783_amd as m
    m.lib()
    return m


def _outputs(sph, tree, n, nsets, static, batch, prm):
    from paper_1309_3783_amd import binding as Bd
    L = Bd.lib()
    ctx = tree.ctx
    tree._in = batch.as_input()
    build = L.sph_build_cells_static if static else L.sph_build_cells
    ctx.check(build(ctx.h, tree.h, C.byref(tree._in), C.byref(prm)), "build")
    ctx.check(L.sph_sort_pairs(ctx.h, tree.h), "sort")
    d = sph.DensityOut(n, "cuda", hash=True)
    f = sph.ForceOut(n, nsets, "cuda", hash=True)
    dc, fc = d.c(), f.c()
    nu, it = C.c_int32(0), C.c_int32(0)
    st = L.sph_solve_h(ctx.h, tree.h, C.byref(dc), C.byref(nu), C.byref(it))
    assert st == sph.SPH_OK, st
    ctx.check(L.sph_force(ctx.h, tree.h, C.byref(fc)), "force")
    torch.cuda.synchronize()
    r = {k: getattr(d, k).cpu().numpy() for k in ("rho", "drho_dh", "nw", "dnw_dh", "nngb", "hash", "h")}
    r.update({"f_" + k: getattr(f, k).cpu().numpy() for k in ("ax", "ay", "az", "dudt", "vsig", "S", "nforce",
                                                                "hash", "sums")})
    return r


def test_static_scratch_matches_allocating_build(sph):
    ctx = sph.Context(0)
    prm = sph.params(flags=sph.SPH_FLAG_PAIR_HASH, h_slack=0.5)
    tree_s = sph.Tree(ctx, workspace=False)     # its memory: the static scratch
    for k, n in enumerate([60000, 17000]):       # two calls, the second smaller
        sets = [sphinputs.plummer_mixture(n, 90 + k, velocity=True, snap=False),
                sphinputs.uniform(n // 7, 95 + k, velocity=True)]
        batch = sph.batch_from_sets(sets)
        ref = _outputs(sph, sph.Tree(ctx, workspace=False), batch.n, batch.nsets, False, batch, prm)
        got = _outputs(sph, tree_s, batch.n, batch.nsets, True, batch, prm)
        for key in ref:
            assert np.array_equal(ref[key], got[key]), (n, key)


def test_static_scratch_limits(sph):
    from paper_1309_3783_amd import binding as Bd
    L = Bd.lib()
    ctx = sph.Context(0)
    prm = sph.params()
    # too large for the scratch: refused before any work
    big = sph.batch_from_sets([sphinputs.uniform(400000, 97)])
    t = sph.Tree(ctx, workspace=False)
    t._in = big.as_input()
    assert L.sph_build_cells_static(ctx.h, t.h, C.byref(t._in), C.byref(prm)) == sph.SPH_E_CAPACITY
    # a second tree takes the scratch over: the first one's calls fail
    small = sph.batch_from_sets([sphinputs.uniform(5000, 98)])
    t1, t2 = sph.Tree(ctx, workspace=False), sph.Tree(ctx, workspace=False)
    t1._in = small.as_input()
    t2._in = small.as_input()
    assert L.sph_build_cells_static(ctx.h, t1.h, C.byref(t1._in), C.byref(prm)) == sph.SPH_OK
    assert L.sph_build_cells_static(ctx.h, t2.h, C.byref(t2._in), C.byref(prm)) == sph.SPH_OK
    assert L.sph_sort_pairs(ctx.h, t1.h) == sph.SPH_E_STATE
    assert L.sph_sort_pairs(ctx.h, t2.h) == sph.SPH_OK
    torch.cuda.synchronize()
