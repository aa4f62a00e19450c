"""Served mode: a request loop with continuous batching over the C-ABI.

Requests (independent particle sets) arrive over time.  The scheduler keeps
a queue of arrived requests and an executor with several lanes; a lane runs
one batch at a time.  Whenever a lane is free it admits the queued requests
that fit the device-memory budget (sph_footprint per request, summed over
everything in flight) and launches them as one batch, so requests that
arrive while others are on the GPU join as soon as a lane and memory free
up, and the lanes' device work overlaps.  A request too large for the free
memory waits while smaller ones behind it go first (head-of-line bypass),
until it has been bypassed `max_bypass` times; then the queue waits for it.

The GPU executor gives each lane its own HIP stream, context, tree and
output buffers: the host builds one lane's cells while the other lane's
graph (Newton passes, ghost, force, sums) runs.  Trees stay on the device
from the build to the force.  Latency = completion - arrival.  Every set
gets its own cells and tasks and every particle sums in an order fixed by
its own set's tree, so a request's results are bitwise the same alone and
in any batch.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    ps: object              # ParticleSet-like (numpy arrays, caller order)
    t_start: float = -1.0
    t_done: float = -1.0
    pairs: float = 0.0
    batch_size: int = 0
    result: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.ps.n

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Scheduler:
    """Admission, queueing and bookkeeping; the executor does the work."""

    def __init__(self, executor, budget_bytes: int, footprint, max_batch: int = 64, max_bypass: int = 4):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.footprint = footprint
        self.max_batch = max_batch
        self.max_bypass = max_bypass
        self.in_use = 0
        self.skips: dict = {}
        self.log: list = []

    def admit(self, queue: collections.deque) -> list:
        chosen, free = [], self.budget - self.in_use
        for r in list(queue):
            if len(chosen) >= self.max_batch:
                break
            fp = self.footprint(r)
            if fp > self.budget:
                raise RuntimeError(f"request {r.rid} ({r.n} particles) exceeds the whole budget")
            if fp <= free:
                chosen.append(r)
                free -= fp
            elif r is queue[0] and not chosen:
                self.skips[r.rid] = self.skips.get(r.rid, 0) + 1
                if self.skips[r.rid] > self.max_bypass:
                    break                 # stop bypassing: wait for the head
        for r in chosen:
            queue.remove(r)
        return chosen

    def run(self, requests: list) -> list:
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = collections.deque(reqs)
        queue: collections.deque = collections.deque()
        self.ex.start()
        while pending or queue or self.ex.busy():
            now = self.ex.now()
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            for lane, batch in self.ex.completed():
                t = self.ex.now()
                for r in batch:
                    r.t_done = t
                self.in_use -= sum(self.footprint(r) for r in batch)
                progressed = True
            while queue:
                lane = self.ex.free_lane()
                if lane is None:
                    break
                chosen = self.admit(queue)
                if not chosen:
                    break
                t = self.ex.now()
                for r in chosen:
                    r.t_start = t
                    r.batch_size = len(chosen)
                self.in_use += sum(self.footprint(r) for r in chosen)
                self.log.append((t, len(chosen), self.in_use))
                self.ex.launch(lane, chosen)
                progressed = True
            if not progressed:
                self.ex.wait(pending[0].arrival if pending else None)
        return reqs


class GpuExecutor:
    """Lanes = HIP streams with their own context, tree and buffers."""

    def __init__(self, prm=None, k_iter: int = 24, lanes: int = 2, keep_results: bool = False, device=0):
        import torch
        from . import binding as B
        from . import pipeline as P
        self.B, self.P, self.torch = B, P, torch
        self.prm = prm or B.params()
        self.k_iter = k_iter
        self.keep = keep_results
        self.lanes = []
        for _ in range(lanes):
            st = torch.cuda.Stream(device)
            ctx = B.Context(device, stream=st)
            self.lanes.append({"stream": st, "ctx": ctx, "tree": B.Tree(ctx), "reqs": None, "event": None})
        self.t0 = time.perf_counter()

    def start(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def busy(self) -> bool:
        return any(l["reqs"] for l in self.lanes)

    def free_lane(self):
        for i, l in enumerate(self.lanes):
            if not l["reqs"]:
                return i
        return None

    def launch(self, i, reqs):
        torch, B, P = self.torch, self.B, self.P
        l = self.lanes[i]
        with torch.cuda.stream(l["stream"]):
            l["batch"] = B.batch_from_sets([r.ps for r in reqs])
            l["out"] = P.Outputs(l["batch"].n, l["batch"].nsets)
            P.launch_graph(l["tree"], l["batch"], self.prm, l["out"], self.k_iter)
            ev = torch.cuda.Event()
            ev.record(l["stream"])
        l["event"], l["reqs"] = ev, reqs

    def completed(self):
        torch, P = self.torch, self.P
        done = []
        for i, l in enumerate(self.lanes):
            if l["reqs"] and l["event"].query():
                with torch.cuda.stream(l["stream"]):
                    P.finish_graph(l["tree"], l["batch"], self.prm, l["out"], self.k_iter)
                    l["stream"].synchronize()
                    sums = l["out"].f.sums.view(-1, 8).cpu().numpy()
                    for s, r in enumerate(l["reqs"]):
                        r.pairs = float(sums[s, 6]) / 2.0
                        if self.keep:
                            r.result = {k: P.per_set(l["batch"], getattr(l["out"].d, k), s)
                                        for k in ("rho", "h", "nngb", "nw")}
                            r.result.update({k: P.per_set(l["batch"], getattr(l["out"].f, k), s)
                                             for k in ("ax", "ay", "az", "dudt", "nforce")})
                done.append((i, l["reqs"]))
                l["reqs"], l["event"], l["batch"], l["out"] = None, None, None, None
        return done

    def wait(self, next_arrival):
        time.sleep(2e-5)


class FakeExecutor:
    """Simulated clock and service times (for testing the scheduler on a CPU):
    a batch takes `base + per_particle * N` seconds on its lane."""

    def __init__(self, lanes: int = 2, base: float = 1e-3, per_particle: float = 2e-9):
        self.lanes = [None] * lanes
        self.base, self.per = base, per_particle
        self.t = 0.0

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def busy(self):
        return any(l is not None for l in self.lanes)

    def free_lane(self):
        for i, l in enumerate(self.lanes):
            if l is None:
                return i
        return None

    def launch(self, i, reqs):
        n = sum(r.n for r in reqs)
        self.lanes[i] = (self.t + self.base + self.per * n, reqs)
        for r in reqs:
            r.pairs = 25.0 * r.n

    def completed(self):
        out = []
        for i, l in enumerate(self.lanes):
            if l is not None and l[0] <= self.t:
                out.append((i, l[1]))
                self.lanes[i] = None
        return out

    def wait(self, next_arrival):
        ends = [l[0] for l in self.lanes if l is not None]
        cands = ends + ([next_arrival] if next_arrival is not None else [])
        if cands:
            self.t = max(self.t, min(cands))


def summary(reqs: list) -> dict:
    lat = np.array([r.latency for r in reqs]) * 1e3
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    pairs = sum(r.pairs for r in reqs)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "requests": len(reqs), "span_s": span,
            "requests_per_s": len(reqs) / span, "pair_interactions_per_s": 2.0 * pairs / span,
            "mean_batch": float(np.mean([r.batch_size for r in reqs]))}
