"""One GPU's share of a set decomposed over 8 GPUs (2 x 2 x 2 blocks of the
top grid): the particles it owns plus the halo, the layer of top cells
around its block (at least the largest h thick, periodic).  Halo particles
are read-only neighbours whose density comes from their owner (here: the
FP64 oracle on the whole set, rounded to FP32).  The owned particles'
density and force must equal the oracle's on the whole set, to the full bar.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import _inputs as I  # noqa: E402

import oracle  # noqa: E402
import sphinputs  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from _checks import FORCE_TOL, RHO_TOL  # noqa: E402


@pytest.fixture(scope="module")
def sph():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1309_3783_amd as m
    m.lib()
    return m


def share_of(ps, lo, edge, halo):
    """Indices of the particles of block [lo, lo + edge)^3 and of its halo
    (within `halo` of the block, periodic), as (owned mask over the share,
    index array into ps)."""
    pos = ps.pos()
    d = np.mod(pos - lo + halo, 1.0)          # block + halo -> [0, edge + 2 halo)
    inside = np.all(d < edge + 2 * halo, axis=1)
    idx = np.nonzero(inside)[0]
    own = np.all((d[idx] >= halo) & (d[idx] < edge + halo), axis=1)
    return own, idx


def subset(ps, idx):
    return sphinputs.ParticleSet(ps.x[idx], ps.y[idx], ps.z[idx], ps.m[idx], ps.u[idx], ps.vx[idx], ps.vy[idx],
                                 ps.vz[idx], ps.h0[idx], ps.box)


def test_share_fixed_h_matches_whole_set(sph):
    ps = sphinputs.lattice(40, 0.1, 33, velocity=True, snap=False)
    ps, h = I.fixed_h_case(ps)
    rd, rf = I.oracle_reference(ps, h)
    ctx = sph.Context(0)
    for blk in [(0.0, 0.0, 0.0), (0.5, 0.0, 0.5)]:
        own, idx = share_of(ps, np.array(blk), 0.5, 0.125)
        # halo / owned = ((0.5 + 2 * 0.125)^3 - 0.5^3) / 0.5^3 = 2.375 at this size
        assert abs((~own).sum() / own.sum() - 2.375) < 0.1
        sub = subset(ps, idx)
        batch = sph.batch_from_sets([sub], h=[h[idx]])
        tree = sph.Tree(ctx)
        tree.build_cells(batch, sph.params(flags=sph.SPH_FLAG_PAIR_HASH))
        assert tree.stats()["top_grid"] == 8              # top cell edge 0.125 = the halo's thickness
        owned = torch.as_tensor(own.astype(np.uint8), device="cuda")
        rho = torch.as_tensor(rd["rho"][idx].astype(np.float32), device="cuda")
        drho = torch.as_tensor(rd["drho_dh"][idx].astype(np.float32), device="cuda")
        tree.set_halo(owned, rho, drho)
        tree.sort_pairs()
        d = sph.DensityOut(sub.n, "cuda", hash=True)
        f = sph.ForceOut(sub.n, 1, "cuda", hash=True)
        tree.density(d)
        tree.force(f)
        torch.cuda.synchronize()
        t = idx[own]
        o = np.nonzero(own)[0]
        # the oracle on the share (its own particle numbering, which the pair
        # hashes use), with the halo densities of the whole set
        hs = h[idx]
        sd = oracle.density(sub.x, sub.y, sub.z, hs, sub.m, sub.box, targets=o)
        sf = oracle.force(sub.x, sub.y, sub.z, hs, sub.m, sub.vx, sub.vy, sub.vz, sub.u, rd["rho"][idx],
                          rd["drho_dh"][idx], sub.box, targets=o)
        # the share holds every neighbour of an owned particle: the same
        # values as on the whole set
        assert np.array_equal(sd["nngb"][o], rd["nngb"][t]) and np.array_equal(sf["nforce"][o], rf["nforce"][t])
        assert np.allclose(sd["rho"][o], rd["rho"][t], rtol=1e-13, atol=0)
        assert np.allclose(sf["ax"][o], rf["ax"][t], rtol=1e-11, atol=1e-12 * rf["S"][t].max())
        assert np.array_equal(d.nngb.cpu().numpy()[o], sd["nngb"][o])
        assert np.array_equal(d.hash.cpu().numpy().view(np.uint64)[o], sd["hash"][o])
        rel = np.abs(d.rho.cpu().numpy()[o] - rd["rho"][t]) / rd["rho"][t]
        assert rel.max() <= RHO_TOL, rel.max()
        assert np.array_equal(f.nforce.cpu().numpy()[o], rf["nforce"][t])
        assert np.array_equal(f.hash.cpu().numpy().view(np.uint64)[o], sf["hash"][o])
        S = rf["S"][t]
        for k in ("ax", "ay", "az"):
            err = np.abs(getattr(f, k).cpu().numpy()[o] - rf[k][t]) / S
            assert err.max() <= FORCE_TOL, (k, err.max())
        # the per-set sums cover the owned particles only: their force
        # neighbour count
        s = f.sums.cpu().numpy()
        assert s[6] == float(rf["nforce"][t].sum())


def test_share_solves_owned_h_only(sph):
    """h solved on the share: owned particles are solved, halo particles keep
    the h they came with; the oracle accepts the owned h (N_w within 48 +-
    0.5 in FP64, evaluated on the whole set) and reproduces their density."""
    ps = sphinputs.lattice(40, 0.1, 34, velocity=True, snap=False)
    h_ref = I.f32(I.solved_h(ps))
    rd = oracle.density(ps.x, ps.y, ps.z, h_ref, ps.m, ps.box)
    own, idx = share_of(ps, np.array([0.5, 0.5, 0.0]), 0.5, 0.125)
    sub = subset(ps, idx)
    ctx = sph.Context(0)
    h_in = h_ref[idx].copy()
    h_in[own] = sub.h0[own]                      # owned: from the first guess; halo: as given
    batch = sph.batch_from_sets([sub], h=[h_in])
    tree = sph.Tree(ctx)
    owned = torch.as_tensor(own.astype(np.uint8), device="cuda")
    rho = torch.as_tensor(rd["rho"][idx].astype(np.float32), device="cuda")
    drho = torch.as_tensor(rd["drho_dh"][idx].astype(np.float32), device="cuda")
    d = sph.DensityOut(sub.n, "cuda")
    d.h.copy_(torch.as_tensor(np.float32(-1.0) * np.ones(sub.n, np.float32), device="cuda"))
    st, nu, it = sph.solve_with_rebuild(tree, batch, sph.params(h_slack=0.5), d, halo=(owned, rho, drho))
    assert st == sph.SPH_OK and nu == 0
    torch.cuda.synchronize()
    hg = d.h.cpu().numpy()
    assert np.all(hg[~own] == -1.0)               # halo entries not written
    o = np.nonzero(own)[0]
    t = idx[o]
    # the whole set with the share's solved h for its owned particles
    hw = h_ref.copy()
    hw[t] = hg[o]
    w = oracle.density(ps.x, ps.y, ps.z, hw, ps.m, ps.box, targets=t)
    assert np.abs(w["nw"][t] - 48.0).max() <= 0.5 + 1e-3
    rel = np.abs(d.rho.cpu().numpy()[o] - w["rho"][t]) / w["rho"][t]
    assert rel.max() <= RHO_TOL
