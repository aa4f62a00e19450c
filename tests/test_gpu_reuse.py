"""GPU parity of a tree reused over time steps (sph_refresh_cells).

Section II-C keeps the sorted indices over several steps until the cells
must be made again.  A refreshed tree keeps the build's cells, cell order
and list order while the particles move; the sweeps reach twice the set's
displacement bound further and the h the cells support shrinks by as much.
Each case builds on one state, moves the particles (FP64, wrapped into the
box, off the 2^-24 grid), refreshes, and compares density and force with
the oracle on the moved state at a fixed h (oracle solve, untied at 1e-6):
pair sets and counts exact (splitmix64 hashes: every pair met exactly
once), density 1e-5, force 1e-4 of S_i.  Also: the refresh is refused once
the displacement eats the cells' margin, and a leapfrog run that reuses the
tree follows the run that rebuilds every step.
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

from _checks import check_density, check_force, check_sums, at_gpu_h  # noqa: E402


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


def moved(ps, dt):
    """The state after x += dt v in FP64, wrapped into the box."""
    q = sphinputs.ParticleSet(np.mod(ps.x + dt * ps.vx, ps.box), np.mod(ps.y + dt * ps.vy, ps.box),
                              np.mod(ps.z + dt * ps.vz, ps.box), ps.m, ps.u, ps.vx, ps.vy, ps.vz, ps.h0, ps.box,
                              dict(ps.meta))
    return q


def results(sph, tree, n):
    dout = sph.DensityOut(n, "cuda", hash=True)
    tree.density(dout)
    fout = sph.ForceOut(n, 1, "cuda", hash=True)
    tree.force(fout)
    torch.cuda.synchronize()
    d = {k: getattr(dout, k).cpu().numpy() for k in ("rho", "drho_dh", "nw", "dnw_dh", "nngb", "h")}
    d["hash"] = dout.hash.cpu().numpy().view(np.uint64)
    f = {k: getattr(fout, k).cpu().numpy() for k in ("ax", "ay", "az", "dudt", "vsig", "S", "nforce")}
    f["hash"] = fout.hash.cpu().numpy().view(np.uint64)
    f["sums"] = fout.sums[:8].cpu().numpy()
    return d, f


def shifted(ps, s):
    """The set translated by s along the diagonal (wrapped)."""
    return sphinputs.ParticleSet(np.mod(ps.x + s, ps.box), np.mod(ps.y + s, ps.box), np.mod(ps.z + s, ps.box),
                                 ps.m, ps.u, ps.vx, ps.vy, ps.vz, ps.h0, ps.box, dict(ps.meta))


CASES = {
    # 24^3 jittered lattice, |v| <= 0.17: each step moves a particle up to
    # ~0.1 h, a fifth of the spacing, so neighbours change order along the
    # pair axes; translated so that rows sit next to the faces and cross the
    # periodic boundary
    "lattice": (lambda: shifted(sphinputs.lattice(24, 0.1, 7, velocity=True, snap=False), 0.0195),
                [0.03, 0.03], 0.5),
    # clumpy mixture, h over ~3 decades, several levels of cells; steps sized
    # to the small h of the clump cores (the displacement bound is the set's
    # largest, met by every particle)
    "clumpy": (lambda: sphinputs.plummer_mixture(20000, 43, n_clumps=6, snap=False, velocity=True),
               [5e-5, 5e-5], 0.5),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_refresh_matches_oracle(sph, ctx, name):
    make, dts, slack = CASES[name]
    ps0 = make()
    print(f"\n[reuse] {name}: n {ps0.n}, steps {dts}, h slack {slack}", flush=True)
    prm = sph.params(flags=sph.SPH_FLAG_PAIR_HASH, h_slack=slack)
    _, h0 = I.fixed_h_case(ps0)
    tree = sph.Tree(ctx)
    tree.build_cells(sph.batch_from_sets([ps0], h=[h0]), prm)
    tree.sort_pairs()
    st0 = tree.stats()
    ps = ps0
    for dt in dts:
        ps = moved(ps, dt)
    crossed = int(np.sum(np.abs(ps.x - ps0.x) > 0.5 * ps.box))
    _, h = I.fixed_h_case(ps)
    # intermediate states refreshed too: the displacement bound adds up
    q = ps0
    for dt in dts[:-1]:
        q = moved(q, dt)
        assert tree.refresh(sph.batch_from_sets([q], h=[h0]))
    assert tree.refresh(sph.batch_from_sets([ps], h=[h]))
    st = tree.stats()
    assert (st["cells"], st["tasks"], st["sorted_entries"]) == (st0["cells"], st0["tasks"], st0["sorted_entries"])
    g_d, g_f = results(sph, tree, ps.n)
    rd, rf = I.oracle_reference(ps, h)
    check_density(ps, h, g_d, rd)
    check_force(ps, g_f, rf)
    check_sums(ps, g_f, rf)
    # a fresh build of the moved state meets the same pairs
    tree2 = sph.Tree(ctx)
    tree2.build_cells(sph.batch_from_sets([ps], h=[h]), prm)
    tree2.sort_pairs()
    b_d, b_f = results(sph, tree2, ps.n)
    assert np.array_equal(b_d["hash"], g_d["hash"]) and np.array_equal(b_f["hash"], g_f["hash"])
    e = float((np.abs(g_d["rho"] - rd["rho"]) / rd["rho"]).max())
    print(f"[reuse] {name}: levels {st['levels']}, crossed the boundary {crossed}, rho rel {e:.2e}", flush=True)
    if name == "lattice":
        assert crossed > 0


def test_refresh_then_solve(sph, ctx):
    """solve_h on a refreshed tree, checked at the h the GPU solved."""
    ps0 = sphinputs.lattice(20, 0.2, 9, velocity=True, snap=False)
    prm = sph.params(h_slack=0.5)
    tree = sph.Tree(ctx)
    d0 = sph.DensityOut(ps0.n, "cuda")
    st, _, _ = sph.solve_with_rebuild(tree, sph.batch_from_sets([ps0]), prm, d0)
    assert st == sph.SPH_OK
    ps = moved(ps0, 0.04)
    b = sph.batch_from_sets([ps], h=[d0.h.cpu().numpy()])
    d = sph.DensityOut(ps.n, "cuda")
    builds = tree.builds
    st, nu, it = sph.solve_with_rebuild(tree, b, prm, d, refresh=True)
    assert st == sph.SPH_OK and nu == 0
    assert tree.builds == builds and tree.refreshes >= 1        # no new build
    f = sph.ForceOut(ps.n, 1, "cuda")
    tree.force(f)
    torch.cuda.synchronize()
    gd = {k: getattr(d, k).cpu().numpy() for k in ("rho", "nw", "nngb", "h")}
    gf = {k: getattr(f, k).cpu().numpy() for k in ("ax", "ay", "az", "nforce")}
    k, e = at_gpu_h(ps, gd, gf)
    print(f"\n[reuse] solve on a refreshed tree: {it} Newton passes, {k} compared, {e} near a cutoff", flush=True)


def test_refresh_refused_past_the_margin(sph, ctx):
    ps0 = sphinputs.lattice(24, 0.1, 11, velocity=True, snap=False)
    prm = sph.params()
    _, h0 = I.fixed_h_case(ps0)
    tree = sph.Tree(ctx)
    tree.build_cells(sph.batch_from_sets([ps0], h=[h0]), prm)
    tree.sort_pairs()
    L0 = 1.0 / tree.stats()["top_grid"]
    # one particle moves by the whole margin of the top cells
    ps = moved(ps0, 0.0)
    ps.x = ps.x.copy()
    ps.x[123] = np.mod(ps.x[123] + 0.5 * (L0 - h0.max()) + 1e-3, 1.0)
    assert not tree.refresh(sph.batch_from_sets([ps], h=[h0]))
    with pytest.raises(sph.SphError):
        tree.density(sph.DensityOut(ps.n, "cuda"))                 # left unbuilt
    # building again gives the right answer
    _, h = I.fixed_h_case(ps, h0)
    tree.build_cells(sph.batch_from_sets([ps], h=[h]), sph.params(flags=sph.SPH_FLAG_PAIR_HASH))
    tree.sort_pairs()
    g_d, g_f = results(sph, tree, ps.n)
    rd, rf = I.oracle_reference(ps, h)
    check_density(ps, h, g_d, rd)


def test_refresh_rejects_another_layout(sph, ctx):
    a = sphinputs.uniform(3000, 5)
    tree = sph.Tree(ctx)
    tree.build_cells(sph.batch_from_sets([a]))
    tree.sort_pairs()
    with pytest.raises(sph.SphError):
        tree.refresh(sph.batch_from_sets([sphinputs.uniform(3001, 5)]))


def test_leapfrog_reuse_follows_rebuild(sph, ctx):
    from paper_1309_3783_amd.integrate import Leapfrog
    ps = sphinputs.lattice(16, 0.1, 13, velocity=True, snap=False)
    out = {}
    for reuse in (False, True):
        b = sph.batch_from_sets([ps])
        # fixed h: a Newton solve may stop on either side of its tolerance
        # when the sums round differently, which would hide the comparison
        lf = Leapfrog(ctx, b, sph.params(h_slack=0.5), solve_h=False, reuse=reuse)
        lf.run(0.06, dt=0.01)
        torch.cuda.synchronize()
        out[reuse] = ({k: getattr(b, k).double().cpu().numpy() for k in ("x", "y", "z", "vx", "vy", "vz", "u")},
                      getattr(lf.tree, "refreshes", 0), lf.tree.builds)
    a, r0, b0 = out[False]
    c, r1, b1 = out[True]
    print(f"\n[reuse] leapfrog 6 steps: rebuild every step {b0} builds; reuse {b1} builds + {r1} refreshes",
          flush=True)
    assert r0 == 0 and r1 >= 3 and b1 < b0
    for k in ("x", "y", "z"):
        d = np.abs(a[k] - c[k])
        d = np.minimum(d, 1.0 - d)
        assert d.max() <= 1e-6, (k, d.max())
    vs = max(np.abs(a[k]).max() for k in ("vx", "vy", "vz"))
    for k in ("vx", "vy", "vz"):
        assert np.abs(a[k] - c[k]).max() <= 1e-5 * vs, k
    assert np.abs(a["u"] - c["u"]).max() <= 1e-5 * np.abs(a["u"]).max()


def test_refresh_batched_graph_replayed(sph, ctx):
    """Several uneven sets in one tree: the graph pipeline on the first
    state, then the sets move, the tree is refreshed and the same graph is
    replayed (no new capture); every set checked at the h the GPU solved."""
    from paper_1309_3783_amd import pipeline as P
    sizes = [3100, 12000, 5400, 21000, 2600]
    sets = [sphinputs.plummer_mixture(n, 1700 + k, velocity=True, snap=False) for k, n in enumerate(sizes)]
    prm = sph.params(h_slack=0.5)
    tree = sph.Tree(ctx)
    b0 = sph.batch_from_sets(sets)
    out0 = P.Outputs(b0.n, b0.nsets)
    P.run_graph(tree, b0, prm, out0, 24)
    torch.cuda.synchronize()
    caps = tree.stats()["graph_captures"]
    h0 = [P.per_set(b0, out0.d.h, s).copy() for s in range(len(sets))]
    moved_sets = [moved(ps, 2e-5) for ps in sets]
    b1 = sph.batch_from_sets(moved_sets, h=h0)
    assert tree.refresh(b1)
    out1 = out0            # the same output buffers: the captured graph applies as it is
    tree.run_graph(24, out1.d, out1.f, out1.status)
    torch.cuda.synchronize()
    P.finish_graph(tree, b1, prm, out1, 24)
    torch.cuda.synchronize()
    assert tree.stats()["graph_captures"] == caps          # replayed, not captured again
    excl = 0
    for s, ps in enumerate(moved_sets):
        r = {k: P.per_set(b1, getattr(out1.d, k), s) for k in ("rho", "h", "nngb", "nw")}
        r.update({k: P.per_set(b1, getattr(out1.f, k), s) for k in ("ax", "ay", "az", "nforce")})
        k, e = at_gpu_h(ps, r, r)
        excl += e
        assert k + e == ps.n
    print(f"\n[reuse] refreshed batch of {len(sets)} sets through the replayed graph: {excl} near a cutoff", flush=True)


def test_refresh_keeps_the_halo(sph, ctx):
    """One GPU's share (owned block + halo of one top cell): built, moved,
    refreshed, the halo's densities set again; the owned particles' density
    and force equal the oracle's on the whole moved set."""
    from test_gpu_share import share_of, subset
    from _checks import RHO_TOL, FORCE_TOL
    import oracle
    ps0 = sphinputs.lattice(40, 0.1, 35, velocity=True, snap=False)
    own, idx = share_of(ps0, np.array([0.0, 0.5, 0.0]), 0.5, 0.125)
    _, h0 = I.fixed_h_case(ps0)
    tree = sph.Tree(ctx)
    prm = sph.params(flags=sph.SPH_FLAG_PAIR_HASH)
    owned = torch.as_tensor(own.astype(np.uint8), device="cuda")
    rd0, _ = I.oracle_reference(ps0, h0)
    tree.build_cells(sph.batch_from_sets([subset(ps0, idx)], h=[h0[idx]]), prm)
    tree.set_halo(owned, torch.as_tensor(rd0["rho"][idx].astype(np.float32), device="cuda"),
                  torch.as_tensor(rd0["drho_dh"][idx].astype(np.float32), device="cuda"))
    tree.sort_pairs()
    ps = moved(ps0, 0.01)
    _, h = I.fixed_h_case(ps, h0)
    rd, rf = I.oracle_reference(ps, h)
    sub = subset(ps, idx)
    assert tree.refresh(sph.batch_from_sets([sub], h=[h[idx]]))
    tree.set_halo(owned, torch.as_tensor(rd["rho"][idx].astype(np.float32), device="cuda"),
                  torch.as_tensor(rd["drho_dh"][idx].astype(np.float32), device="cuda"))
    d = sph.DensityOut(sub.n, "cuda")
    f = sph.ForceOut(sub.n, 1, "cuda")
    tree.density(d)
    tree.force(f)
    torch.cuda.synchronize()
    o = np.nonzero(own)[0]
    t = idx[o]
    rel = np.abs(d.rho.cpu().numpy()[o] - rd["rho"][t]) / rd["rho"][t]
    assert rel.max() <= RHO_TOL, rel.max()
    assert np.array_equal(d.nngb.cpu().numpy()[o], rd["nngb"][t])
    assert np.array_equal(f.nforce.cpu().numpy()[o], rf["nforce"][t])
    S = rf["S"][t]
    for k in ("ax", "ay", "az"):
        err = np.abs(getattr(f, k).cpu().numpy()[o] - rf[k][t]) / S
        assert err.max() <= FORCE_TOL, (k, err.max())
    print(f"\n[reuse] refreshed share: {o.size} owned, {idx.size - o.size} halo, rho rel {rel.max():.2e}", flush=True)


def test_refresh_on_the_static_workspace(sph, ctx):
    """A tree on the no-allocation scratch refreshes in place and gives what
    a tree on its own workspace gives after the same refresh, bit for bit."""
    ps0 = sphinputs.plummer_mixture(9000, 77, velocity=True, snap=False)
    ps = moved(ps0, 1e-4)
    prm = sph.params(flags=sph.SPH_FLAG_PAIR_HASH, h_slack=0.5)
    res = []
    for static in (False, True):
        tree = sph.Tree(ctx)
        b0 = sph.batch_from_sets([ps0])
        if static:
            tree.build_cells_static(b0, prm)
        else:
            tree.build_cells(b0, prm)
        tree.sort_pairs()
        assert tree.refresh(sph.batch_from_sets([ps]))
        res.append(results(sph, tree, ps.n))
    for a, b in zip(res[0], res[1]):
        for k in a:
            assert np.array_equal(a[k], b[k]), k


def test_refresh_two_top_cells_per_side(sph, ctx):
    """Two top cells per side: particles that move just past the far face of
    the top cell they were built in (and past the periodic face) keep
    offsets from that cell's origin on the right periodic image."""
    ps0 = sphinputs.uniform(1000, 61, velocity=True, snap=False)
    # particles close to the faces x = 1/2 and x = 1 move out through them
    near = (np.mod(ps0.x, 0.5) > 0.49)
    vx = ps0.vx.copy()
    vx[near] = 0.1
    ps0 = sphinputs.ParticleSet(ps0.x, ps0.y, ps0.z, ps0.m, ps0.u, vx, ps0.vy, ps0.vz, ps0.h0, ps0.box,
                                dict(ps0.meta))
    prm = sph.params(flags=sph.SPH_FLAG_PAIR_HASH, h_slack=0.5)
    _, h0 = I.fixed_h_case(ps0)
    tree = sph.Tree(ctx)
    tree.build_cells(sph.batch_from_sets([ps0], h=[h0]), prm)
    tree.sort_pairs()
    assert tree.stats()["top_grid"] == 2
    ps = moved(ps0, 0.15)
    crossed = int(np.sum(near & (np.floor(ps.x / 0.5) != np.floor(ps0.x / 0.5))))
    assert crossed >= 5, crossed
    _, h = I.fixed_h_case(ps, h0)
    assert tree.refresh(sph.batch_from_sets([ps], h=[h]))
    g_d, g_f = results(sph, tree, ps.n)
    rd, rf = I.oracle_reference(ps, h)
    check_density(ps, h, g_d, rd)
    check_force(ps, g_f, rf)
    print(f"\n[reuse] two top cells per side: {crossed} particles left their top cell", flush=True)
