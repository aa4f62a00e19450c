"""Benchmark: SPH pair interactions per second (density + force) on one MI355X.

One step = the whole hot path over one synthetic particle set already in HBM:
cell build (Morton sort, refinement, task lists) -> per-(cell, axis) sorts ->
Newton solve of h_i with density passes -> ghost -> force -> FP64 sums.
value = 2 P / t_step, P = unordered pairs with r < max(h_i, h_j) at the solved
h (one density and one force interaction each).

Default workload: 1,000,000 particles on a 100^3 lattice jittered by
U(+-0.1) spacings (seed 2), h solved by Newton to 48 +- 0.5.
The same line carries the batched comparison (256 uneven sets in one build
and one HIP graph, autotuned, vs the plain one-set-at-a-time loop) and the
served Poisson stream (p50/p99 latency).  --config multires times the 8M
clumpy set instead; --config sod / sedov time leapfrog time steps of the
paper's shock tube / blast (each step: three kicks, a drift, build, sort, h
solve, force, the Courant step).  Prints ONE JSON line.
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
# Newton passes captured in the batched/served graphs
K_ITER = 24


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
    raise SystemExit(f"unknown config {name}")


# the translation unit of k_density / k_force: its source and every header it
# includes (the counters in profiles/traffic.json hold for these bytes only)
KERNEL_SOURCES = ["paper_1309_3783_amd/csrc/sph_interact.hip", "paper_1309_3783_amd/csrc/sph_impl.h",
                  "paper_1309_3783_amd/csrc/sph_internal.h", "paper_1309_3783_amd/csrc/sph_prims.h",
                  "include/sphcell.h", "paper_1309_3783_amd/build.py"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and on this workload; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash() or d.get("workload") != workload:
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(sets, budget_s=15.0):
    """The FP64 oracle on this host, on a random sample of target particles
    of the same set: h solve, density and force for the targets (the other
    particles keep their first-guess h and the density at it, computed
    untimed beforehand).  Rate = sum over targets of their force neighbours
    (each target's share of 2P) / timed seconds."""
    import oracle
    ps = sets[0]
    rng = np.random.default_rng(0)
    ncores = oracle.num_threads()
    t_prep = time.perf_counter()
    d0 = oracle.density(ps.x, ps.y, ps.z, ps.h0, ps.m, ps.box)
    t_prep = time.perf_counter() - t_prep
    k = 1000
    while True:
        t = np.sort(rng.choice(ps.n, size=min(k, ps.n), replace=False))
        t0 = time.perf_counter()
        h, _ = oracle.solve_h(ps.x, ps.y, ps.z, ps.m, ps.h0, ps.box, targets=t, tol=0.5)
        d = oracle.density(ps.x, ps.y, ps.z, h, ps.m, ps.box, targets=t)
        rho = d0["rho"].copy()
        drho = d0["drho_dh"].copy()
        rho[t] = d["rho"][t]
        drho[t] = d["drho_dh"][t]
        f = oracle.force(ps.x, ps.y, ps.z, h, ps.m, ps.vx, ps.vy, ps.vz, ps.u, rho, drho, ps.box, targets=t)
        dt = time.perf_counter() - t0
        pairs = int(f["nforce"][t].sum())
        if dt >= 0.5 * budget_s or k >= ps.n:
            break
        k = min(ps.n, int(k * min(16.0, max(2.0, budget_s / max(dt, 1e-3)))))
    return {"value": pairs / dt, "unit": "pair interactions/s", "cores": ncores, "kind": "oracle",
            "sample": f"{k} random targets of the same {ps.n}-particle set: FP64 h solve + density + force "
                      f"for the targets ({dt:.1f} s); other particles at their first-guess h with density "
                      f"from an untimed pass ({t_prep:.1f} s)"}


def run(args):
    import torch
    import paper_1309_3783_amd as sph

    sets, cfg = make_workload(args.config)
    log(f"[bench] workload {cfg}")
    dev = "cuda"
    ctx = sph.Context(0)
    stream = ctx.stream
    batch = sph.batch_from_sets(sets, device=dev)
    prm = sph.params(**({"h_slack": args.slack} if args.slack is not None else {}))
    n = batch.n
    dout = sph.DensityOut(n, dev)
    fout = sph.ForceOut(n, batch.nsets, dev)
    tree = sph.Tree(ctx)

    stage = {}

    def record():
        for name, ms in ctx.timings():
            stage.setdefault(name, []).append(ms)

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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        it, nu = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.enable_timing(False)
    # stage events of the timed steps (recorded on the context stream,
    # read once after the loop)
    record()
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
    log(f"[bench] newton iterations {it} (incl. rebuilds)")

    ach = P * OPS_FORCE / (force_ms / 1e3)
    traffic = measured_traffic("k_force", cfg["workload"])
    roof = {"kernel": "k_force", "bound": "alu", "achieved": ach / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "Tlane-op/s", "frac": ach / VALU_PEAK, "traffic": traffic,
            "launch_ms": force_ms, "ops_per_pair": OPS_FORCE, "pairs_per_launch": P}
    # the HBM side: the kernel's measured bytes per launch against the peak
    # and against what a plain device copy reaches on this GPU
    copy_tbs = copy_bandwidth()
    roof["hbm"] = {"copy_TBps": copy_tbs, "peak_TBps": HBM_PEAK / 1e12,
                   "k_force_TBps": traffic / (force_ms / 1e3) / 1e12 if traffic else None}
    if traffic:
        roof["hbm"]["frac_of_peak"] = roof["hbm"]["k_force_TBps"] * 1e12 / HBM_PEAK
        roof["hbm"]["frac_of_copy"] = roof["hbm"]["k_force_TBps"] / copy_tbs
    out = {"metric": "pair interactions/sec (density+force), batched vs plain; p50/p99 latency",
           "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": cfg,
           "kernel_pairs_per_s": 2.0 * P / ((force_ms + dens_ms) / 1e3),
           "pairs_P": P, "newton_iterations": it, "unconverged": nu,
           "stages_ms": {k: float(np.mean(v)) for k, v in stage.items()},
           "tree": st, "roofline": roof}
    if args.config == "plain" and not args.quick:
        out["batched"] = bench_batched(sph)
        log(f"[bench] batched {out['batched']['value']:.3g} pairs/s vs plain loop "
            f"{out['batched']['plain_loop']['value']:.3g}")
        out["served"] = bench_served(sph)
        log(f"[bench] served p50 {out['served']['p50_ms']:.2f} ms p99 {out['served']['p99_ms']:.2f} ms")
    if not args.skip_cpu and args.config == "plain":
        log("[bench] timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(sets, budget_s=args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    return out


def plain_loop(sph, ctx, sets, prm):
    """The same sets one at a time: one build / solve / force per set."""
    import torch
    singles = [sph.batch_from_sets([s]) for s in sets]
    douts = [sph.DensityOut(s.n, "cuda") for s in sets]
    fouts = [sph.ForceOut(s.n, 1, "cuda") for s in sets]
    tree = sph.Tree(ctx)
    for b, d, f in zip(singles[:4], douts, fouts):      # warm-up
        sph.solve_with_rebuild(tree, b, prm, d)
        tree.force(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, d, f in zip(singles, douts, fouts):
        sph.solve_with_rebuild(tree, b, prm, d)
        tree.force(f)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    P = sum(float(f.sums[6].item()) / 2.0 for f in fouts)
    return {"value": 2 * P / t, "ms_per_step": t * 1e3, "pairs_P": P}


def bench_batched(sph, n_sets=256, steps=3):
    """Many uneven sets in one batch (one build, one graph) vs the plain loop."""
    import torch
    from paper_1309_3783_amd import autotune, pipeline as P
    import sphinputs
    t = time.perf_counter()
    sets = sphinputs.batch_sets(n_sets)
    log(f"[bench] batched workload: {n_sets} sets, {sum(s.n for s in sets)} particles "
        f"({time.perf_counter() - t:.1f} s to generate)")
    ctx = sph.Context(0)
    batch = sph.batch_from_sets(sets)
    best = autotune.tune(ctx, batch, k_iter=K_ITER, reps=1, label="batched", use_cache=False, log=log)
    prm = sph.params(**best)
    tree = sph.Tree(ctx)
    out = P.Outputs(batch.n, batch.nsets)
    P.run_graph(tree, batch, prm, out, K_ITER)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fallbacks = 0
    for _ in range(steps):
        fallbacks += P.run_graph(tree, batch, prm, out, K_ITER)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    Pp = P.pair_count(out)
    plain = plain_loop(sph, ctx, sets, sph.params())
    return {"workload": "batched_256_sets", "n": batch.n, "sets": n_sets, "n_range": [2000, 200000],
            "value": 2 * Pp / (ms / 1e3), "unit": "pair interactions/s", "ms_per_step": ms, "pairs_P": Pp,
            "autotuned": best, "eager_fallbacks": fallbacks, "plain_loop": plain,
            "speedup_vs_plain": (2 * Pp / (ms / 1e3)) / plain["value"]}


def bench_served(sph, n_req=400, pool_size=24, load=0.7, h_slack=0.2):
    """Poisson request stream, N log-uniform in [1e4, 2e6], continuous batching."""
    from paper_1309_3783_amd import serve as S
    import sphinputs
    rng = np.random.default_rng(5)
    t = time.perf_counter()
    _, pool_n = sphinputs.arrivals(pool_size, 1.0)
    pool = [sphinputs.plummer_mixture(int(n), 5000 + k) for k, n in enumerate(pool_n)]
    log(f"[bench] served pool: {pool_size} sets, {sum(p.n for p in pool)} particles "
        f"({time.perf_counter() - t:.1f} s to generate)")
    # cold starts from the analytic first guess: room for h to grow (0.3
    # measured no better: the latencies vary more between runs than between
    # 0.2 and 0.3)
    prm = sph.params(h_slack=h_slack)
    budget = 64 << 30
    ex = S.GpuExecutor(prm, k_iter=K_ITER, lanes=2)

    def fp(r):
        return sph.footprint(r.n, prm)

    # saturation: everything queued at t = 0
    idx = rng.integers(0, pool_size, size=48)
    burst = [S.Request(i, 0.0, pool[k]) for i, k in enumerate(idx)]
    S.Scheduler(ex, budget, fp, max_batch=16).run(burst[:8])          # warm-up
    sat = S.summary(S.Scheduler(ex, budget, fp, max_batch=16).run(burst))["requests_per_s"]
    rate = load * sat
    gaps = rng.exponential(1.0 / rate, size=n_req)
    arr = np.cumsum(gaps) - gaps[0]
    idx = rng.integers(0, pool_size, size=n_req)
    reqs = [S.Request(i, float(a), pool[k]) for i, (a, k) in enumerate(zip(arr, idx))]
    summ = S.summary(S.Scheduler(ex, budget, fp, max_batch=16).run(reqs))
    summ.update({"saturation_requests_per_s": sat, "arrival_rate_per_s": rate, "load": load,
                 "n_range": [10000, 2000000], "pool_sets": pool_size, "budget_bytes": budget})
    return summ


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Bytes read + written per second by a plain 1 GiB device copy (TB/s)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * nbytes / t / 1e12


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, to scale the HBM byte counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def bench_steps(args):
    """Time steps of the paper's validation set-ups: the shock tube (780,448 +
    197,173 particles standing in for 800,000 + 200,000) or the blast on the
    101^3 lattice.  W untimed steps, then K timed ones, each at the Courant
    step of the current forces."""
    import torch
    import paper_1309_3783_amd as sph
    from paper_1309_3783_amd import integrate
    import sphinputs
    ps = sphinputs.sod() if args.config == "sod" else sphinputs.sedov(101)
    ctx = sph.Context(0)
    batch = sph.batch_from_sets([ps])
    lf = integrate.Leapfrog(ctx, batch)
    for _ in range(args.warmup):
        lf.step(lf.cfl_dt())
    torch.cuda.synchronize()
    t0, e0 = lf.t, lf.energy()
    pairs = 0.0
    t = time.perf_counter()
    for _ in range(args.steps):
        lf.step(lf.cfl_dt())
        pairs += float(lf.f.sums[6].item()) / 2.0
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    e1 = lf.energy()
    ms = el * 1e3 / args.steps
    log(f"[bench] {args.config}: {args.steps} steps in {el:.3f} s ({ms:.2f} ms/step), t {t0:.4g} -> {lf.t:.4g}, "
        f"dE/E {(e1 - e0) / e0:.2e}")
    if args.config == "sod":
        cfg = {"workload": "sod_shock_tube_1M", "n": ps.n, "n_left": ps.meta["n_left"],
               "n_right": ps.meta["n_right"], "rho": [1.0, ps.meta["rho_right"]], "P": [1.0, 0.1795]}
    else:
        cfg = {"workload": "sedov_blast_101^3", "n": ps.n, "E": 100.0, "hot_particles": 33, "P0": 1e-5}
    cfg.update({"step": "kick-drift-kick, Courant 0.3", "h": "Newton to N_w = 48 +- 0.5"})
    return {"metric": "pair interactions/sec (density+force) within leapfrog time steps", "value": 2 * pairs / el,
            "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": cfg,
            "sim_time": [t0, lf.t], "energy_drift": (e1 - e0) / e0, "cpu_baseline": None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="plain", choices=["plain", "multires", "sod", "sedov"])
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only (no batched/served)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--slack", type=float, default=None, help="h slack of the cell decisions (default: library's)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    out = bench_steps(args) if args.config in ("sod", "sedov") else run(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
