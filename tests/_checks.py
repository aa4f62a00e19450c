"""Parity checks shared by the GPU test files: run the HIP path through the
C-ABI at a given h and compare with the FP64 oracle element by element.

Bar: pair sets and neighbour counts bit-exact (counts and splitmix64 pair
hashes), density <= 1e-5 relative, force <= 1e-4 of the per-particle term
scale S_i, momentum/energy sums within 1e-5 of sum m S.
"""
import numpy as np
import torch

import _inputs as I

RHO_TOL = 1e-5
FORCE_TOL = 1e-4
SUM_TOL = 1e-5


def run_fixed(sph, ctx, sets, hs, flags=0, **prm_kw):
    """build -> sort -> density -> force at the given h; numpy results per set
    (flags: SPH_FLAG_* added to the pair-hash flag)."""
    prm = sph.params(flags=sph.SPH_FLAG_PAIR_HASH | flags, **prm_kw)
    batch = sph.batch_from_sets(sets, h=hs)
    tree = sph.Tree(ctx)
    tree.build_cells(batch, prm)
    tree.sort_pairs()
    n = batch.n
    dout = sph.DensityOut(n, "cuda", hash=True)
    tree.density(dout)
    fout = sph.ForceOut(n, batch.nsets, "cuda", hash=True)
    tree.force(fout)
    torch.cuda.synchronize()
    res = []
    for s in range(batch.nsets):
        a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
        d = {k: getattr(dout, k)[a:b].cpu().numpy() for k in ("rho", "drho_dh", "nw", "dnw_dh", "nngb", "h")}
        d["hash"] = dout.hash[a:b].cpu().numpy().view(np.uint64)
        f = {k: getattr(fout, k)[a:b].cpu().numpy() for k in ("ax", "ay", "az", "dudt", "vsig", "S", "nforce")}
        f["hash"] = fout.hash[a:b].cpu().numpy().view(np.uint64)
        f["sums"] = fout.sums[8 * s:8 * s + 8].cpu().numpy()
        res.append((d, f))
    return res, tree


def check_density(ps, h, g, r):
    assert np.array_equal(g["nngb"], r["nngb"]), "density neighbour counts differ"
    assert np.array_equal(g["hash"], r["hash"]), "density pair sets differ"
    assert np.array_equal(g["h"].astype(np.float64), h)
    rel = np.abs(g["rho"] - r["rho"]) / r["rho"]
    assert rel.max() <= RHO_TOL, f"rho rel err {rel.max():.3g}"
    reln = np.abs(g["nw"] - r["nw"]) / r["nw"]
    assert reln.max() <= RHO_TOL, f"N_w rel err {reln.max():.3g}"
    # derivatives: relative to their own size, floored at their natural
    # size 3 rho / h (their terms have mixed signs, so the value can sit near
    # zero; and where many neighbours sit close to the cutoff the value is
    # many times the natural size)
    e1 = np.abs(g["drho_dh"] - r["drho_dh"]) / np.maximum(3 * r["rho"] / h, np.abs(r["drho_dh"]))
    e2 = np.abs(g["dnw_dh"] - r["dnw_dh"]) / np.maximum(3 * r["nw"] / h, np.abs(r["dnw_dh"]))
    assert e1.max() <= RHO_TOL and e2.max() <= RHO_TOL, (e1.max(), e2.max())


def check_force(ps, g, r, targets=None):
    t = np.arange(ps.n) if targets is None else np.asarray(targets)
    assert np.array_equal(g["nforce"][t], r["nforce"][t]), "force neighbour counts differ"
    assert np.array_equal(g["hash"][t], r["hash"][t]), "force pair sets differ"
    S = r["S"][t]
    for k in ("ax", "ay", "az"):
        err = np.abs(g[k][t] - r[k][t]) / np.maximum(S, 1e-300)
        assert err.max() <= FORCE_TOL, f"{k} err/S {err.max():.3g}"
    vmax = max(np.abs(ps.vx).max(), np.abs(ps.vy).max(), np.abs(ps.vz).max(), 1e-30)
    err = np.abs(g["dudt"][t] - r["dudt"][t]) / np.maximum(S * 2 * np.sqrt(3) * vmax, 1e-300)
    assert err.max() <= FORCE_TOL, f"dudt err {err.max():.3g}"
    assert np.allclose(g["S"][t], S, rtol=RHO_TOL, atol=0)
    assert np.allclose(g["vsig"][t], r["vsig"][t], rtol=RHO_TOL, atol=0)


def check_sums(ps, g, r):
    s = g["sums"]
    scale = float(np.sum(ps.m * r["S"]))
    assert abs(s[4] - scale) <= 1e-5 * scale
    assert np.all(np.abs(s[:3]) <= SUM_TOL * scale), s[:3]
    assert abs(s[3]) <= SUM_TOL * scale, s[3]
    assert s[6] == float(r["nforce"].sum())


def full_check(sph, ctx, ps, h, **kw):
    (g,), tree = run_fixed(sph, ctx, [ps], [h], **kw)
    rd, rf = I.oracle_reference(ps, h)
    check_density(ps, h, g[0], rd)
    check_force(ps, g[1], rf)
    assert g[0]["nngb"].sum() == g[1]["sums"][5]
    check_sums(ps, g[1], rf)
    return g, rd, rf, tree




def at_gpu_h(ps, g_d, g_f=None, n_target=48.0, tol=0.5, alpha=None, targets=None):
    """Check results at a smoothing length the GPU solved for (several h are
    correct: any with |N_w - n_target| <= tol).  The oracle evaluates N_w at
    the GPU's h in FP64 (validity of the answer), then the density -- and the
    force, when given -- at that h, element by element.  Targets with a pair
    within 1e-6 of a cutoff at that h are excluded from the exact set
    comparisons and counted.  g_d / g_f: numpy dicts of the GPU outputs of
    one set (caller order).  Returns (number compared, number excluded)."""
    import oracle
    h = np.asarray(g_d["h"], dtype=np.float32).astype(np.float64)
    t = np.arange(ps.n) if targets is None else np.asarray(targets)
    kw = {} if alpha is None else {"alpha": alpha}
    if g_f is None:
        d = oracle.density(ps.x, ps.y, ps.z, h, ps.m, ps.box, targets=t)
    else:
        # the force needs the densities of every force neighbour of the targets
        nb = np.arange(ps.n) if targets is None else \
            np.nonzero(oracle.force_neighbours(ps.x, ps.y, ps.z, h, t, ps.box))[0]
        d = oracle.density(ps.x, ps.y, ps.z, h, ps.m, ps.box, targets=nb)
        f = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, d["rho"], d["drho_dh"], ps.box,
                         targets=t, **kw)
    # the GPU's answer is valid: N_w at its h within tol (FP32 rounding of N_w
    # on the GPU side moves the converged value by ~1e-5 relative)
    assert np.abs(d["nw"][t] - n_target).max() <= tol + 1e-3, np.abs(d["nw"][t] - n_target).max()
    tie = oracle.near_cutoff(ps.x, ps.y, ps.z, h, ps.box, targets=t)[t]
    k = t[~tie]
    assert np.array_equal(np.asarray(g_d["nngb"])[k], d["nngb"][k]), "density neighbour counts differ"
    rel = np.abs(np.asarray(g_d["rho"])[t] - d["rho"][t]) / d["rho"][t]
    w = int(t[np.argmax(rel)])
    assert rel.max() <= RHO_TOL, (f"rho rel err {rel.max():.3g} at particle {w}: h {h[w]:.6g} nngb gpu "
                                  f"{np.asarray(g_d['nngb'])[w]} oracle {d['nngb'][w]} rho gpu "
                                  f"{np.asarray(g_d['rho'])[w]:.8g} oracle {d['rho'][w]:.8g} nw gpu "
                                  f"{np.asarray(g_d['nw'])[w]:.8g} oracle {d['nw'][w]:.8g}; "
                                  f"{int((rel > RHO_TOL).sum())} above the bar")
    reln = np.abs(np.asarray(g_d["nw"])[t] - d["nw"][t]) / d["nw"][t]
    assert reln.max() <= RHO_TOL, f"N_w rel err {reln.max():.3g}"
    if g_f is not None:
        assert np.array_equal(np.asarray(g_f["nforce"])[k], f["nforce"][k]), "force neighbour counts differ"
        S = f["S"][t]
        for c in ("ax", "ay", "az"):
            err = np.abs(np.asarray(g_f[c])[t] - f[c][t]) / np.maximum(S, 1e-300)
            assert err.max() <= FORCE_TOL, f"{c} err/S {err.max():.3g}"
    return int(k.size), int(tie.sum())
