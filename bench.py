"""Benchmark: SPH pair interactions per second (density + force) on one MI355X.

One step = the whole hot path over one synthetic particle set already in HBM:
cell build (Morton sort, refinement, task lists) -> per-(cell, axis) sorts ->
Newton solve of h_i with density passes -> ghost -> force -> FP64 sums.
value = 2 P / t_step, P = unordered pairs with r < max(h_i, h_j) at the solved
h (one density and one force interaction each).

Default workload: 1,000,000 particles on a 100^3 lattice jittered by
U(+-0.1) spacings (seed 2), h solved by Newton to 48 +- 0.5.
Options: --config multires (8M clumpy set) / batched (256 sets, batched vs
plain loop).  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK = 256 * 4 * 16 * 2.4e9     # FP32 lane-ops/s, non-packed (39.3e12)
HBM_PEAK = 8.0e12
# algorithmic VALU lane-ops per unordered interacting pair (both sides, one
# distance test each, no compensation terms): see the design notes
OPS_DENSITY = 52.0
OPS_FORCE = 118.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import sphinputs
    if name == "plain":
        ps = sphinputs.lattice(100, 0.1, 2)
        return [ps], {"workload": "jittered_lattice_1M", "n": ps.n, "lattice": "100^3", "jitter": 0.1,
                      "seed": 2, "h": "Newton to N_w = 48 +- 0.5", "box": "periodic unit cube"}
    if name == "multires":
        ps = sphinputs.plummer_mixture(8_000_000, 3)
        return [ps], {"workload": "plummer_mixture_8M", "n": ps.n, "clumps": 64, "bg_frac": 0.2, "seed": 3,
                      "h": "Newton to N_w = 48 +- 0.5"}
    if name == "batched":
        sets = sphinputs.batch_sets(256)
        return sets, {"workload": "batched_256_sets", "n": int(sum(s.n for s in sets)), "sets": 256,
                      "n_range": [2000, 200000], "seeds": "1000+s"}
    raise SystemExit(f"unknown config {name}")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1309_3783_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1309_3783_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(sets, budget_s=20.0):
    """The FP64 oracle on this host: h solve + density + force for a random
    sample of target particles of the same workload."""
    import oracle
    ps = sets[0]
    rng = np.random.default_rng(0)
    ncores = oracle.num_threads()
    k = 2000
    total_pairs = 0
    total_t = 0.0
    h_all = None
    while True:
        t = np.sort(rng.choice(ps.n, size=min(k, ps.n), replace=False))
        t0 = time.perf_counter()
        h, _ = oracle.solve_h(ps.x, ps.y, ps.z, ps.m, ps.h0, ps.box, targets=t, tol=0.5)
        d = oracle.density(ps.x, ps.y, ps.z, h if h_all is None else h, ps.m, ps.box, targets=t)
        t1 = time.perf_counter()
        # force needs rho of the targets' neighbours: use the targets' own
        # values for them (untimed fill); pair counts come from the timed pass
        rho = np.where(d["rho"] > 0, d["rho"], 1.0)
        drho = np.where(d["rho"] > 0, d["drho_dh"], -3.0)
        hh = np.where(d["rho"] > 0, h, ps.h0)
        t2 = time.perf_counter()
        f = oracle.force(ps.x, ps.y, ps.z, hh, ps.m, ps.vx, ps.vy, ps.vz, ps.u, rho, drho, ps.box, targets=t)
        t3 = time.perf_counter()
        total_t += (t1 - t0) + (t3 - t2)
        total_pairs += int(f["nforce"][t].sum())
        if total_t >= budget_s or k >= ps.n:
            break
        k = min(ps.n, int(k * max(2.0, budget_s / max(total_t, 1e-3))))
    return {"value": total_pairs / total_t, "unit": "pair interactions/s", "cores": ncores, "kind": "oracle",
            "sample": f"FP64 oracle h solve + density + force for random target samples of the same set "
                      f"(last sample {k} targets, {total_t:.1f} s timed); each target counts its force "
                      f"neighbours (= its share of 2P)"}


def run(args):
    import torch
    import paper_1309_3783_amd as sph

    sets, cfg = make_workload(args.config)
    log(f"[bench] workload {cfg}")
    dev = "cuda"
    ctx = sph.Context(0)
    stream = ctx.stream
    batch = sph.batch_from_sets(sets, device=dev)
    prm = sph.params()
    n = batch.n
    dout = sph.DensityOut(n, dev)
    fout = sph.ForceOut(n, batch.nsets, dev)
    tree = sph.Tree(ctx)

    def step():
        st, nu, it = sph.solve_with_rebuild(tree, batch, prm, dout)
        if st not in (sph.SPH_OK, sph.SPH_E_NOCONV):
            raise RuntimeError(f"solve failed: status {st}")
        tree.force(fout)
        return it, nu

    for w in range(args.warmup):
        it, nu = step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w}: newton iterations {it}, unconverged {nu}")
    ctx.enable_timing(True)
    stage = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        it, nu = step()
        for name, ms in ctx.timings():
            stage.setdefault(name, []).append(ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.enable_timing(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    sums = fout.sums.view(-1, 8).cpu().numpy()
    P = float(sums[:, 6].sum()) / 2.0
    value = 2.0 * P / (ms_step / 1e3)
    st = tree.stats()
    force_ms = float(np.mean(stage.get("force", [float("nan")])))
    dens_ms = float(np.mean(stage.get("solve", [float("nan")])))
    log(f"[bench] {args.steps} steps: {ms_step:.2f} ms/step, P = {P:.4g}, stages {{"
        + ", ".join(f"{k}: {np.mean(v):.3f}" for k, v in stage.items()) + "}")
    log(f"[bench] tree {st}")

    ach = P * OPS_FORCE / (force_ms / 1e3)
    roof = {"kernel": "k_force", "bound": "alu", "achieved": ach / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "Tlane-op/s", "frac": ach / VALU_PEAK, "traffic": measured_traffic("k_force"),
            "launch_ms": force_ms, "ops_per_pair": OPS_FORCE, "pairs_per_launch": P}
    out = {"metric": "pair interactions/sec (density+force), batched vs plain; p50/p99 latency",
           "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": cfg,
           "kernel_pairs_per_s": 2.0 * P / ((force_ms + dens_ms) / 1e3),
           "pairs_P": P, "newton_iterations": it, "unconverged": nu,
           "stages_ms": {k: float(np.mean(v)) for k, v in stage.items()},
           "tree": st, "roofline": roof}
    if args.config == "batched":
        out["plain_loop"] = plain_loop(sph, ctx, sets, prm, args.steps)
    if not args.skip_cpu:
        log("[bench] timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(sets, budget_s=args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    return out


def plain_loop(sph, ctx, sets, prm, steps):
    """The same sets one at a time (one build/solve/force per set)."""
    import torch
    singles = [sph.batch_from_sets([s]) for s in sets]
    douts = [sph.DensityOut(s.n, "cuda") for s in sets]
    fouts = [sph.ForceOut(s.n, 1, "cuda") for s in sets]
    tree = sph.Tree(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = 0.0
    for b, d, f in zip(singles, douts, fouts):
        sph.solve_with_rebuild(tree, b, prm, d)
        tree.force(f)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    for f in fouts:
        P += float(f.sums[6].item()) / 2.0
    return {"value": 2 * P / t, "ms_per_step": t * 1e3, "pairs_P": P}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="plain", choices=["plain", "multires", "batched"])
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    out = run(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
