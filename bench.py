"""Benchmark: SPH pair interactions per second (density + force) on one MI355X.

One step = the whole hot path over one synthetic particle set already in HBM:
cell build (Morton sort, refinement, task lists) -> per-(cell, axis) sorts ->
Newton solve of h_i with density passes -> ghost -> force -> FP64 sums.
value = 2 P / t_step, P = unordered pairs with r < max(h_i, h_j) at the solved
h (one density and one force interaction each).

Default workload: 1,000,000 particles on a 100^3 lattice jittered by
U(+-0.1) spacings (seed 2), h solved by Newton to 48 +- 0.5.
The same line carries the multi-resolution workload (8,000,000 particles,
64 Plummer clumps + 20% background, h over ~3 decades: the stand-in for the
paper's cosmological volume), the batched comparison (256 uneven sets in one
build and one HIP graph, autotuned, vs the plain one-set-at-a-time loop) and
the served Poisson stream (p50/p99 latency) and one GPU's share of an
8-GPU decomposition (1M owned particles of a 200^3 lattice plus their
read-only halo).  --config multires times only the 8M clumpy set; --config
share only the share; --config sod / sedov time leapfrog time steps of the
paper's shock tube / blast.  Prints ONE JSON line.

Roofline accounting (the interaction kernels are bound by vector ALU work):
algorithmic lane-ops per unordered pair, frozen: density 70, force 125
(one evaluation per unordered pair with compensated accumulators; sqrt
counted as 4), against 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12
FP32 lane-ops/s.  The pairs a launch processes are counted on the device
(sph_last_work: the neighbour counts of the particles each pass evaluated,
halved: an unordered pair is seen from both sides).  The decomposition and
the sorts are priced against HBM: 250 B per particle for the build (keys,
six radix passes, the cell-ordered gather) and 40 B per sorted-list entry
(position and h read, a 20 B record written).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK = 256 * 4 * 16 * 2.4e9     # FP32 lane-ops/s, non-packed (39.3e12)
HBM_PEAK = 8.0e12
OPS_DENSITY = 70.0                   # lane-ops per unordered pair (frozen op table)
OPS_FORCE = 125.0
BUILD_BYTES_PER_PARTICLE = 250.0
SORT_BYTES_PER_ENTRY = 40.0
K_ITER = 24                          # Newton passes captured in the batched/served graphs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import sphinputs
    if name == "plain":
        ps = sphinputs.lattice(100, 0.1, 2)
        return ps, {"workload": "jittered_lattice_1M", "n": ps.n, "lattice": "100^3", "jitter": 0.1,
                    "seed": 2, "h": "Newton to N_w = 48 +- 0.5", "box": "periodic unit cube"}
    if name == "multires":
        ps = sphinputs.plummer_mixture(8_000_000, 3)
        return ps, {"workload": "plummer_mixture_8M", "n": ps.n, "clumps": 64, "bg_frac": 0.2, "seed": 3,
                    "h": "Newton to N_w = 48 +- 0.5", "box": "periodic unit cube"}
    raise SystemExit(f"unknown config {name}")


# the translation unit of k_density / k_force: its source and every header it
# includes (the counters in profiles/traffic.json hold for this code only;
# comments do not count)
KERNEL_SOURCES = ["paper_1309_3783_amd/csrc/sph_interact.hip", "paper_1309_3783_amd/csrc/sph_impl.h",
                  "paper_1309_3783_amd/csrc/sph_internal.h", "paper_1309_3783_amd/csrc/sph_prims.h",
                  "include/sphcell.h", "paper_1309_3783_amd/build.py"]


def _strip_comments(text: str, py: bool) -> str:
    """The code of a source file without its comments and blank lines (the
    hash follows code changes, not edits of the documentation)."""
    import re
    if py:
        lines = [ln.split("#", 1)[0].rstrip() for ln in text.splitlines()]
    else:
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
    return "\n".join(ln for ln in lines if ln.strip())


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_strip_comments(fh.read(), f.endswith(".py")).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and on this workload; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get("workloads", {}).get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ps, gpu_h, gpu_nforce, budget_s=15.0, check_max=20000):
    """The FP64 oracle on this host, on a random sample of target particles
    of the same set: h solve, density and force for the targets (the other
    particles keep their first-guess h and the density at it, computed
    untimed beforehand).  Rate = sum over targets of their force neighbours
    (each target's share of 2 P) / timed seconds.  Untimed afterwards, the
    numerator the GPU line uses is checked on a sample of targets: the
    oracle's force-neighbour counts at the GPU's solved h against the GPU's
    (targets with a pair within 1e-6 of a cutoff at that h left out)."""
    import oracle
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
    # the numerator: force-neighbour counts at the GPU's h, oracle vs GPU
    hg = np.asarray(gpu_h, dtype=np.float32).astype(np.float64)
    tc = np.sort(rng.choice(ps.n, size=min(check_max, ps.n), replace=False))
    nc = oracle.force_neighbours(ps.x, ps.y, ps.z, hg, tc, ps.box)
    nb = np.nonzero(nc)[0]
    dc = oracle.density(ps.x, ps.y, ps.z, hg, ps.m, ps.box, targets=nb)
    fc = oracle.force(ps.x, ps.y, ps.z, hg, ps.m, ps.vx, ps.vy, ps.vz, ps.u, dc["rho"], dc["drho_dh"], ps.box,
                      targets=tc)
    tie = oracle.near_cutoff(ps.x, ps.y, ps.z, hg, ps.box, targets=tc)[tc]
    keep = tc[~tie]
    equal = bool(np.array_equal(np.asarray(gpu_nforce)[keep], fc["nforce"][keep]))
    return {"value": pairs / dt, "unit": "pair interactions/s", "cores": ncores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{k} random targets of the same {ps.n}-particle set: FP64 h solve + density + force "
                      f"for the targets ({dt:.1f} s); other particles at their first-guess h with density "
                      f"from an untimed pass ({t_prep:.1f} s)",
            "pairs_check": {"targets": int(keep.size), "excluded_near_cutoff": int(tie.sum()),
                            "nforce_equal_to_oracle": equal}}


def measure(sph, ps, steps, warmup, prm):
    """K timed steps of the whole path on one set; per-step device times,
    stage times and the work the interaction kernels did."""
    import torch
    ctx = sph.Context(0)
    batch = sph.batch_from_sets([ps])
    n = batch.n
    dout = sph.DensityOut(n, "cuda")
    fout = sph.ForceOut(n, 1, "cuda")
    tree = sph.Tree(ctx)

    def step():
        st, nu, it = sph.solve_with_rebuild(tree, batch, prm, dout)
        if st not in (sph.SPH_OK, sph.SPH_E_NOCONV):
            raise RuntimeError(f"solve failed: status {st}")
        tree.force(fout)
        return it, nu

    for w in range(warmup):
        it, nu = step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w}: newton iterations {it}, unconverged {nu}")
    ctx.enable_timing(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(ctx.stream)
        it, nu = step()
        ev[k][1].record(ctx.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.enable_timing(False)
    stage = {}
    for name, ms in ctx.timings():
        stage.setdefault(name, []).append(ms)
    # the work of the last step (every step repeats the same computation)
    wd, wf = ctx.work()
    rd, rf = ctx.reads()
    step_ms = np.array([a.elapsed_time(b) for a, b in ev])
    sums = fout.sums.view(-1, 8).cpu().numpy()
    return {"ms_per_step": (t1 - t0) * 1e3 / steps, "step_ms": step_ms, "stage": stage,
            "P": float(sums[:, 6].sum()) / 2.0, "work_density": wd, "work_force": wf,
            "reads_density": rd, "reads_force": rf,
            "it": it, "nu": nu, "tree": tree.stats(), "dout": dout, "fout": fout,
            "ws_bytes": int(tree.ws.numel()) if tree.ws is not None else None,
            "ws_peak": tree.workspace_needed()}


def rooflines(m, steps, workload):
    """VALU roofline of both interaction kernels, and the HBM fractions of the
    build and sort stages, from one measurement."""
    st = m["stage"]
    dens = st.get("density_pass", [])
    force = st.get("force", [])
    out = {}
    for name, times, work, ops in (("k_density", dens, m["work_density"], OPS_DENSITY),
                                   ("k_force", force, m["work_force"], OPS_FORCE)):
        if not times:
            continue
        launches = len(times) / steps
        t_step = float(np.sum(times)) / steps            # ms of this kernel per step
        units = work / 2.0                               # unordered-pair units per step
        ach = units * ops / (t_step / 1e3)
        traffic = measured_traffic(name, workload)
        out[name] = {"kernel": name, "bound": "alu", "achieved": ach / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "Tlane-op/s", "frac": ach / VALU_PEAK, "traffic": traffic,
                     "launch_ms": t_step / launches, "launches_per_step": launches, "ms_per_step": t_step,
                     "ops_per_pair": ops, "pairs_per_launch": units / launches}
        if traffic:
            bps = traffic / (t_step / launches / 1e3)
            out[name]["hbm"] = {"TBps": bps / 1e12, "frac_of_peak": bps / HBM_PEAK}
    n = m["tree"]["particles"]
    ent = m["tree"]["sorted_entries"]
    stages = {}
    for name, per in (("build", BUILD_BYTES_PER_PARTICLE * n), ("sort", SORT_BYTES_PER_ENTRY * ent)):
        if name in st:
            t = float(np.mean(st[name])) / 1e3
            stages[name] = {"bound": "hbm", "algorithmic_bytes": per, "ms": t * 1e3,
                            "achieved_TBps": per / t / 1e12, "peak_TBps": HBM_PEAK / 1e12,
                            "frac": per / t / HBM_PEAK}
    return out, stages


def summarize(m, steps):
    step_ms = m["step_ms"]
    return {"ms_per_step": m["ms_per_step"], "step_ms_p50": float(np.percentile(step_ms, 50)),
            "step_ms_p99": float(np.percentile(step_ms, 99)), "pairs_P": m["P"],
            "value": 2.0 * m["P"] / (m["ms_per_step"] / 1e3),
            "newton_iterations": m["it"], "unconverged": m["nu"],
            "stages_ms": {k: float(np.sum(v)) / steps for k, v in m["stage"].items() if k != "start"},
            "tree": m["tree"], "workspace_bytes": m["ws_bytes"], "workspace_peak_bytes": m["ws_peak"]}


def run(args):
    import paper_1309_3783_amd as sph

    ps, cfg = make_workload(args.config)
    log(f"[bench] workload {cfg}")
    prm = sph.params(**({"h_slack": args.slack} if args.slack is not None else {}))
    m = measure(sph, ps, args.steps, args.warmup, prm)
    s = summarize(m, args.steps)
    rl, stages = rooflines(m, args.steps, cfg["workload"])
    log(f"[bench] {args.steps} steps: {s['ms_per_step']:.2f} ms/step (p50 {s['step_ms_p50']:.2f}, "
        f"p99 {s['step_ms_p99']:.2f}), P = {s['pairs_P']:.4g}, stages "
        + ", ".join(f"{k}: {v:.3f}" for k, v in s["stages_ms"].items()))
    for k, r in rl.items():
        log(f"[bench] {k}: {r['launch_ms']:.3f} ms/launch x {r['launches_per_step']:.1f}, "
            f"{r['achieved']:.2f} Tlane-op/s = {100 * r['frac']:.1f}% of VALU peak")
    log(f"[bench] tree {s['tree']}")
    # the dominant interaction kernel of a step carries the roofline object
    dom = max(rl.values(), key=lambda r: r["ms_per_step"])
    roof = dict(dom)
    copy_tbs = copy_bandwidth()
    roof["hbm_copy_TBps"] = copy_tbs
    out = {"metric": "pair interactions/sec (density+force), batched vs plain; p50/p99 latency",
           "value": s["value"], "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": s["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": cfg,
           "step_ms_p50": s["step_ms_p50"], "step_ms_p99": s["step_ms_p99"],
           "kernel_pairs_per_s": 2.0 * s["pairs_P"] / (sum(r["ms_per_step"] for r in rl.values()) / 1e3),
           "pairs_P": s["pairs_P"], "newton_iterations": s["newton_iterations"], "unconverged": s["unconverged"],
           "stages_ms": s["stages_ms"], "tree": s["tree"], "workspace_bytes": s["workspace_bytes"],
           "workspace_peak_bytes": s["workspace_peak_bytes"], "roofline": roof, "rooflines": rl,
           "stage_hbm": stages}
    if not args.skip_cpu:
        log("[bench] timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(ps, m["dout"].h.cpu().numpy(), m["fout"].nforce.cpu().numpy(),
                                           budget_s=args.cpu_budget)
        log(f"[bench] oracle {out['cpu_baseline']['value']:.3g} pairs/s on {out['cpu_baseline']['cores']} cores, "
            f"pair counts equal: {out['cpu_baseline']['pairs_check']}")
    else:
        out["cpu_baseline"] = None
    if args.config == "plain" and not args.quick:
        out["reuse"] = bench_reuse(sph, ps, dt=1e-3)
    del m
    if args.config == "plain" and not args.quick:
        out["multires"] = bench_multires(sph, args)
        out["share"] = bench_share(sph)
        out["batched"] = bench_batched(sph)
        log(f"[bench] batched {out['batched']['value']:.3g} pairs/s vs plain loop "
            f"{out['batched']['plain_loop']['value']:.3g} (tuned parameters "
            f"{out['batched']['plain_loop_tuned']['value']:.3g})")
        out["served"] = bench_served(sph)
        sv = out["served"]
        log(f"[bench] served p50 {sv['p50_ms']:.2f} ms p99 {sv['p99_ms']:.2f} ms at {sv['load']:.0%} load; "
            f"saturated {sv['saturation_pair_interactions_per_s']:.3g} pairs/s "
            f"(mean batch {sv['saturation_mean_batch']:.1f}) vs plain one at a time "
            f"{sv['plain_same_stream']['pair_interactions_per_s']:.3g}")
    return out


def bench_multires(sph, args, steps=3, warmup=1):
    """The 8M clumpy mixture (h over ~3 decades), with the same accounting."""
    import torch
    t = time.perf_counter()
    ps, cfg = make_workload("multires")
    log(f"[bench] multires workload generated in {time.perf_counter() - t:.1f} s")
    m = measure(sph, ps, steps, warmup, sph.params())
    s = summarize(m, steps)
    rl, stages = rooflines(m, steps, cfg["workload"])
    log(f"[bench] multires {steps} steps: {s['ms_per_step']:.2f} ms/step, P = {s['pairs_P']:.4g}, "
        + ", ".join(f"{k}: {v:.3f}" for k, v in s["stages_ms"].items()))
    for k, r in rl.items():
        log(f"[bench] multires {k}: {r['ms_per_step']:.2f} ms/step, {100 * r['frac']:.1f}% of VALU peak")
    res = {"config": cfg, "steps": steps, "warmup": warmup, "unit": "pair interactions/s", **s,
           "rooflines": rl, "stage_hbm": stages}
    if not args.skip_cpu:
        log("[bench] timing the FP64 oracle on the host (multires sample)")
        res["cpu_baseline"] = cpu_baseline(ps, m["dout"].h.cpu().numpy(), m["fout"].nforce.cpu().numpy(),
                                           budget_s=args.cpu_budget, check_max=5000)
    del m
    torch.cuda.empty_cache()
    res["reuse"] = bench_reuse(sph, ps, dt=2e-6)
    return res


def with_velocities(ps, seed=17, vmax=0.1):
    """A copy of the set with velocities uniform in [-vmax, vmax] (FP32)."""
    import sphinputs
    rng = np.random.default_rng(seed)
    v = rng.uniform(-vmax, vmax, size=(ps.n, 3)).astype(np.float32).astype(np.float64)
    return sphinputs.ParticleSet(ps.x, ps.y, ps.z, ps.m, ps.u, v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(),
                                 ps.h0, ps.box, dict(ps.meta))


def bench_reuse(sph, ps, dt, steps=10):
    """Cells and sorted lists reused over time steps (Section II-C) against a
    build and sort every step, on the same sequence of states: the set drifts
    by x += dt v between steps (sph_drift; velocities uniform in [-0.1, 0.1]
    where the set has none) and each step solves h from the previous step's h
    and computes the forces.  dt is chosen so the displacement bound stays
    inside the cells' margin for all the steps (the refresh path would
    otherwise fall back to a build, which it counts)."""
    import dataclasses
    import torch
    if not np.any(ps.vx):
        ps = with_velocities(ps)
    prm = sph.params()
    out = {"dt": dt, "steps": steps}
    for reuse in (False, True):
        ctx = sph.Context(0)
        b = sph.batch_from_sets([ps])
        d = sph.DensityOut(b.n, "cuda")
        f = sph.ForceOut(b.n, 1, "cuda")
        tree = sph.Tree(ctx)
        st, _, _ = sph.solve_with_rebuild(tree, b, prm, d)
        tree.force(f)
        builds0 = tree.builds
        torch.cuda.synchronize()
        ctx.enable_timing(True)
        t0 = time.perf_counter()
        its = 0
        for _ in range(steps):
            sph.drift(ctx, b, dt)
            b.h.copy_(d.h)
            st, nu, it = sph.solve_with_rebuild(tree, b, prm, d, refresh=reuse)
            if st not in (sph.SPH_OK, sph.SPH_E_NOCONV):
                raise RuntimeError(f"solve failed: status {st}")
            its += it
            tree.force(f)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.enable_timing(False)
        stage = {}
        for name, ms in ctx.timings():
            if name != "start":
                stage[name] = stage.get(name, 0.0) + ms / steps
        key = "reuse" if reuse else "rebuild"
        out[key] = {"ms_per_step": (t1 - t0) * 1e3 / steps, "builds": tree.builds - builds0,
                    "refreshes": getattr(tree, "refreshes", 0), "newton_passes": its / steps, "stages_ms": stage}
        del tree, d, f, b
        torch.cuda.empty_cache()
    out["speedup"] = out["rebuild"]["ms_per_step"] / out["reuse"]["ms_per_step"]
    log(f"[bench] reuse over {steps} steps of dt {dt:g}: {out['reuse']['ms_per_step']:.2f} ms/step "
        f"({out['reuse']['refreshes']} refreshes, {out['reuse']['builds']} builds; refresh "
        f"{out['reuse']['stages_ms'].get('refresh', 0.0):.3f} ms) vs build + sort every step "
        f"{out['rebuild']['ms_per_step']:.2f} ms/step (build {out['rebuild']['stages_ms'].get('build', 0.0):.3f}, "
        f"sort {out['rebuild']['stages_ms'].get('sort', 0.0):.3f} ms)")
    return out


def bench_share(sph, steps=10, warmup=2):
    """One GPU's share of an 8-GPU decomposition at its real size: a 200^3
    jittered lattice (8M particles, h solved whole on this GPU first, standing
    in for the other GPUs' work) cut into 2 x 2 x 2 blocks; the share is the
    block [0, 1/2)^3 (1M owned particles) plus the halo, one top cell of the
    whole set around it (periodic), whose h, density and d rho/dh come from
    the whole-set run (what a halo exchange delivers).  A step on the share:
    build, sort, h solve of the owned particles, force of the owned ones."""
    import torch
    import sphinputs
    ps = sphinputs.lattice(200, 0.1, 2)
    ctx = sph.Context(0)
    whole = sph.batch_from_sets([ps])
    d = sph.DensityOut(ps.n, "cuda")
    tree = sph.Tree(ctx)
    st, nu, it = sph.solve_with_rebuild(tree, whole, sph.params(), d)
    edge = 1.0 / tree.stats()["top_grid"]                # the halo: one top cell of the whole set
    h_all, rho_all, drho_all = d.h.cpu().numpy(), d.rho.cpu().numpy(), d.drho_dh.cpu().numpy()
    del tree, d, whole
    torch.cuda.empty_cache()
    pos = ps.pos()
    dd = np.mod(pos + edge, 1.0)
    idx = np.nonzero(np.all(dd < 0.5 + 2 * edge, axis=1))[0]
    own = np.all((dd[idx] >= edge) & (dd[idx] < 0.5 + edge), axis=1)
    sub = sphinputs.ParticleSet(ps.x[idx], ps.y[idx], ps.z[idx], ps.m[idx], ps.u[idx], ps.vx[idx], ps.vy[idx],
                                ps.vz[idx], np.where(own, ps.h0[idx], h_all[idx]), ps.box)
    batch = sph.batch_from_sets([sub])
    owned = torch.as_tensor(own.astype(np.uint8), device="cuda")
    rho = torch.as_tensor(rho_all[idx], device="cuda")
    drho = torch.as_tensor(drho_all[idx], device="cuda")
    tree = sph.Tree(ctx)
    dout = sph.DensityOut(sub.n, "cuda")
    fout = sph.ForceOut(sub.n, 1, "cuda")
    prm = sph.params()

    def step():
        st, nu, it = sph.solve_with_rebuild(tree, batch, prm, dout, halo=(owned, rho, drho))
        if st not in (sph.SPH_OK, sph.SPH_E_NOCONV):
            raise RuntimeError(f"share solve failed: status {st}")
        tree.force(fout)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    pairs = float(fout.sums[6].item())          # force neighbours of the owned particles (their share of 2 P)
    log(f"[bench] share: {int(own.sum())} owned + {int((~own).sum())} halo particles, {ms:.2f} ms/step, "
        f"{pairs / (ms / 1e3):.3g} pairs/s")
    return {"workload": "lattice_200^3_share_1_of_8", "owned": int(own.sum()), "halo": int((~own).sum()),
            "halo_thickness": edge, "steps": steps, "ms_per_step": ms, "unit": "pair interactions/s",
            "value": pairs / (ms / 1e3), "owned_force_pairs": pairs,
            "note": "pair interactions of the owned particles (each one's force neighbours) per second"}


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
    """Many uneven sets in one batch (one build, one graph) vs the plain loop,
    with the default parameters and with the autotuned ones."""
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
    plain_tuned = plain_loop(sph, ctx, sets, prm)
    val = 2 * Pp / (ms / 1e3)
    return {"workload": "batched_256_sets", "n": batch.n, "sets": n_sets, "n_range": [2000, 200000],
            "value": val, "unit": "pair interactions/s", "ms_per_step": ms, "pairs_P": Pp,
            "autotuned": best, "eager_fallbacks": fallbacks, "plain_loop": plain, "plain_loop_tuned": plain_tuned,
            "speedup_vs_plain": val / plain["value"], "speedup_vs_plain_tuned": val / plain_tuned["value"]}


def bench_served(sph, n_req=1000, n_warm=50, n_plain=300, pool_size=24, load=0.7, h_slack=0.2, lanes=4):
    """Poisson request stream, N log-uniform in [1e4, 2e6], continuous batching
    over `lanes` executor lanes (4: against 2 and 3, the highest saturation
    rate and the lowest latency at 70% of it);
    beside it the first n_plain requests of the same stream run one at a time
    back to back (the plain path).  The served results are checked against the
    oracle by the GPU tests (every request there), not here."""
    import torch
    from paper_1309_3783_amd import serve as S
    import sphinputs
    rng = np.random.default_rng(5)
    t = time.perf_counter()
    _, pool_n = sphinputs.arrivals(pool_size, 1.0)
    pool = [sphinputs.plummer_mixture(int(n), 5000 + k) for k, n in enumerate(pool_n)]
    log(f"[bench] served pool: {pool_size} sets, {sum(p.n for p in pool)} particles "
        f"({time.perf_counter() - t:.1f} s to generate)")
    prm = sph.params(h_slack=h_slack)
    budget = 64 << 30
    ex = S.GpuExecutor(prm, k_iter=K_ITER, lanes=lanes)

    def fp(r):
        return sph.footprint(r.n, prm)

    # saturation: everything queued at t = 0
    idx = rng.integers(0, pool_size, size=48)
    burst = [S.Request(i, 0.0, pool[k]) for i, k in enumerate(idx)]
    S.Scheduler(ex, budget, fp, max_batch=16).run(burst[:8])          # warm-up
    sat_summ = S.summary(S.Scheduler(ex, budget, fp, max_batch=16).run(burst))
    sat = sat_summ["requests_per_s"]
    rate = load * sat
    total = n_warm + n_req
    gaps = rng.exponential(1.0 / rate, size=total)
    arr = np.cumsum(gaps) - gaps[0]
    idx = rng.integers(0, pool_size, size=total)
    reqs = [S.Request(i, float(a), pool[k]) for i, (a, k) in enumerate(zip(arr, idx))]
    S.Scheduler(ex, budget, fp, max_batch=16).run(reqs)
    summ = S.summary(reqs[n_warm:])
    summ.update({"saturation_requests_per_s": sat,
                 "saturation_pair_interactions_per_s": sat_summ["pair_interactions_per_s"],
                 "saturation_mean_batch": sat_summ["mean_batch"], "arrival_rate_per_s": rate, "load": load,
                 "warmup_requests": n_warm, "n_range": [10000, 2000000], "pool_sets": pool_size,
                 "budget_bytes": budget})
    # the plain path on the same stream: one request at a time, no batching
    ctx = sph.Context(0)
    tree = sph.Tree(ctx)
    pairs = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs[n_warm:n_warm + n_plain]:
        b = sph.batch_from_sets([r.ps])
        d = sph.DensityOut(r.n, "cuda")
        f = sph.ForceOut(r.n, 1, "cuda")
        sph.solve_with_rebuild(tree, b, prm, d)
        tree.force(f)
        pairs += float(f.sums[6].item()) / 2.0
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    summ["plain_same_stream"] = {"requests": n_plain, "seconds": tp, "pair_interactions_per_s": 2 * pairs / tp,
                                 "requests_per_s": n_plain / tp}
    summ["saturation_speedup_vs_plain"] = summ["saturation_pair_interactions_per_s"] / (2 * pairs / tp)
    ex.close()
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
    ap.add_argument("--config", default="plain", choices=["plain", "multires", "share", "sod", "sedov"])
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only (no multires/batched/served)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--slack", type=float, default=None, help="h slack of the cell decisions (default: library's)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (the library has no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)
    if args.config == "share":
        import paper_1309_3783_amd as sph
        out = bench_share(sph, steps=args.steps, warmup=args.warmup)
    else:
        out = bench_steps(args) if args.config in ("sod", "sedov") else run(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
