"""Autotuner for the batched pipeline.

Times the graph pipeline over a grid of launch and decomposition parameters
on the actual batch (or a sample of it) and keeps the fastest:
  * n_split        -- leaf size (split count of Section III-B, 400 by default)
  * blocks_per_cu  -- resident persistent blocks (4 wavefronts each) per CU (0: as many as fit)
  * max_replicas   -- lanes per target particle for small chunks
  * h_slack        -- room left for h to grow before the cells must be
                      rebuilt (more room: fewer rebuilds, larger cells)
  * top_coarsen    -- top grid one level coarser than the largest allowed
                      (larger top cells, split further where dense)
Results are cached in a JSON table keyed by a workload signature (number of
sets and log2 of the mean set size).
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

from . import binding as B
from . import pipeline as P

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned.json")

GRID = {"n_split": [200, 400, 800], "blocks_per_cu": [0, 3, 4], "max_replicas": [4, 16], "h_slack": [0.2, 0.3],
        "top_coarsen": [0, 1]}


def signature(batch: B.Batch, label: str = "") -> str:
    mean = batch.n / max(batch.nsets, 1)
    return f"{label}:sets{batch.nsets}:logn{int(round(math.log2(max(mean, 1))))}"


def load_table() -> dict:
    if os.path.exists(TABLE):
        try:
            with open(TABLE) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            # unreadable or half-written table: tune again
            return {}
    return {}


def save_table(tab: dict) -> None:
    tmp = TABLE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(tab, fh, indent=1, sort_keys=True)
    os.replace(tmp, TABLE)


def tune(ctx: B.Context, batch: B.Batch, base: dict | None = None, k_iter: int = 24, reps: int = 2,
         grid: dict | None = None, label: str = "", use_cache: bool = True, log=None) -> dict:
    import torch
    sig = signature(batch, label)
    tab = load_table() if use_cache else {}
    if use_cache and sig in tab:
        return tab[sig]["best"]
    grid = grid or GRID
    base = dict(base or {})
    keys = list(grid)
    tree = B.Tree(ctx)
    out = P.Outputs(batch.n, batch.nsets)
    results = []
    for vals in itertools.product(*(grid[k] for k in keys)):
        cand = dict(zip(keys, vals))
        prm = B.params(**base, **cand)
        times = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.run_graph(tree, batch, prm, out, k_iter)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = sorted(times[1:])[len(times[1:]) // 2]
        results.append((t, cand))
        if log:
            log(f"[autotune] {cand}: {t * 1e3:.2f} ms")
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    if use_cache:
        tab[sig] = {"best": best, "ms": results[0][0] * 1e3,
                    "all": [{"ms": t * 1e3, **c} for t, c in results]}
        save_table(tab)
    return best
