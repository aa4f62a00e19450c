"""Whole-pipeline drivers over the C-ABI: eager (build -> sort -> solve_h ->
force) and graph mode (build -> sort -> one HIP graph holding the Newton
passes, ghost, force and sums).  Argument marshalling only."""
from __future__ import annotations

import numpy as np

from . import binding as B


class Outputs:
    """Density and force outputs plus the device status words of a batch
    ([0] unconverged, [1] rebuild, then per set: unconverged, rebuild)."""

    def __init__(self, n: int, nsets: int, device="cuda", hash=False):
        import torch
        self.d = B.DensityOut(n, device, hash=hash)
        self.f = B.ForceOut(n, nsets, device, hash=hash)
        self.status = torch.zeros(2 + 2 * max(nsets, 1), dtype=torch.int32, device=device)


DENSITY_FIELDS = ("rho", "drho_dh", "nw", "dnw_dh", "nngb", "h", "hash")
FORCE_FIELDS = ("ax", "ay", "az", "dudt", "vsig", "S", "nforce", "hash")


def sub_batch(batch: B.Batch, sets, h_full) -> B.Batch:
    """The listed sets of a batch as a new batch, with smoothing lengths taken
    from h_full (caller order of the full batch)."""
    import torch
    idx = [(int(batch.offsets[s]), int(batch.offsets[s + 1])) for s in sets]

    def cat(t):
        return torch.cat([t[a:b] for a, b in idx]) if idx else t[:0]

    sizes = [b - a for a, b in idx]
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return B.Batch(cat(batch.x), cat(batch.y), cat(batch.z), cat(h_full), cat(batch.m), cat(batch.u),
                   cat(batch.vx), cat(batch.vy), cat(batch.vz), off, batch.box[list(sets)])


def run_eager(tree: B.Tree, batch: B.Batch, prm, out: Outputs):
    st, nu, it = B.solve_with_rebuild(tree, batch, prm, out.d)
    if st not in (B.SPH_OK, B.SPH_E_NOCONV):
        raise B.SphError(st, "solve_h")
    tree.force(out.f)
    return it, nu


def launch_graph(tree: B.Tree, batch: B.Batch, prm, out: Outputs, k_iter: int):
    """build + sort (these synchronise the stream) and enqueue the graph;
    returns without waiting for the graph."""
    tree.build_cells(batch, prm)
    tree.sort_pairs()
    tree.run_graph(k_iter, out.d, out.f, out.status)


def _copy_set(out: Outputs, batch: B.Batch, s: int, sub_out: Outputs, sub: B.Batch, k: int):
    a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
    c, d = int(sub.offsets[k]), int(sub.offsets[k + 1])
    for f in DENSITY_FIELDS:
        dst, src = getattr(out.d, f), getattr(sub_out.d, f)
        if dst is not None and src is not None:
            dst[a:b].copy_(src[c:d])
    for f in FORCE_FIELDS:
        dst, src = getattr(out.f, f), getattr(sub_out.f, f)
        if dst is not None and src is not None:
            dst[a:b].copy_(src[c:d])
    out.f.sums[8 * s:8 * s + 8].copy_(sub_out.f.sums[8 * k:8 * k + 8])


def failing_sets(out: Outputs, nsets: int) -> list:
    st = out.status.cpu().numpy()
    if st[0] == 0 and st[1] == 0:
        return []
    return [s for s in range(nsets) if st[2 + 2 * s] != 0 or st[3 + 2 * s] != 0]


def finish_graph(tree: B.Tree, batch: B.Batch, prm, out: Outputs, k_iter: int, max_rounds: int = 4):
    """After the stream has been synchronised: the sets whose h did not
    converge in the graph's fixed number of passes, or outgrew their cells,
    are rebuilt from the h they reached and run again through the graph,
    together (the graph keeps sets independent: per-set status words), for
    up to max_rounds rounds; a set still failing then finishes with the eager
    calls on its own.  Results are copied into the batch outputs; the other
    sets keep theirs, so every set ends exactly as it would alone.
    Returns the number of set re-runs."""
    bad = failing_sets(out, batch.nsets)
    if not bad:
        return 0
    reruns = 0
    # one auxiliary tree per main tree, and the outputs of each round, are
    # kept from call to call: a batch that needs the same re-run every step
    # allocates once
    aux = getattr(tree, "_aux", None)
    if aux is None:
        aux = tree._aux = B.Tree(tree.ctx)
    cache = tree.__dict__.setdefault("_aux_out", {})
    hashed = out.d.hash is not None
    cur_batch, cur_out, ids = batch, out, list(range(batch.nsets))
    for r in range(max_rounds):
        sub = sub_batch(cur_batch, bad, cur_out.d.h)
        key = (sub.n, sub.nsets, hashed)
        if r not in cache or cache[r][0] != key:
            cache[r] = (key, Outputs(sub.n, sub.nsets, hash=hashed))
        sub_out = cache[r][1]
        launch_graph(aux, sub, prm, sub_out, k_iter)
        aux.ctx.stream.synchronize()
        reruns += len(bad)
        ids = [ids[s] for s in bad]
        still = set(failing_sets(sub_out, sub.nsets))
        for k, s in enumerate(ids):
            if k not in still:
                _copy_set(out, batch, s, sub_out, sub, k)
        if not still:
            return reruns
        cur_batch, cur_out = sub, sub_out
        bad = sorted(still)
    ids = [ids[s] for s in bad]
    for k0, s in zip(bad, ids):
        one = sub_batch(cur_batch, [k0], cur_out.d.h)
        one_out = Outputs(one.n, 1, hash=out.d.hash is not None)
        run_eager(aux, one, prm, one_out)
        _copy_set(out, batch, s, one_out, one, 0)
        reruns += 1
    return reruns


def run_graph(tree: B.Tree, batch: B.Batch, prm, out: Outputs, k_iter: int = 24):
    launch_graph(tree, batch, prm, out, k_iter)
    tree.ctx.sync()
    return finish_graph(tree, batch, prm, out, k_iter)


def pair_count(out: Outputs) -> float:
    s = out.f.sums.view(-1, 8).cpu().numpy()
    return float(s[:, 6].sum()) / 2.0


def per_set(batch: B.Batch, t, s: int) -> np.ndarray:
    a, b = int(batch.offsets[s]), int(batch.offsets[s + 1])
    return t[a:b].cpu().numpy()
