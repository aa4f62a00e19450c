"""Served mode: a request loop with continuous batching over the C-ABI.

Requests (independent particle sets) arrive over time.  The scheduler keeps
a queue of arrived requests and an executor with several lanes; a lane runs
one batch at a time.  Whenever a lane is free it admits the queued requests
that fit the device-memory budget and launches them as one batch, so
requests that arrive while others are on the GPU join as soon as a lane and
memory free up, and the lanes' device work overlaps.  A request too large
for the free memory waits while smaller ones behind it go first
(head-of-line bypass), until it has been bypassed `max_bypass` times; then
the queue waits for it.

Memory: a batch is charged its workspace estimate (sph_workspace_size over
its particles and sets, the `footprint` of the requests summed); a lane
keeps the workspace of its tree between batches (grow-only), and what it
keeps is charged too, running or idle (`retained`), so the budget bounds
the device memory the lanes really hold.

The GPU executor gives each lane its own HIP stream, context, tree (with
its workspace), output buffers and worker thread: the upload, the build
with its few read-backs, the sort and the graph launch of a batch run on
the lane's thread, so the host work of one lane overlaps the device work of
the other and the scheduler thread only admits and books.  Trees stay on
the device from the build to the force.  Latency = completion - arrival.
Every set gets its own cells and tasks and every particle sums in an order
fixed by its own set's tree, so a request's results are bitwise the same
alone and in any batch.
"""
from __future__ import annotations

import collections
import queue as _queue
import threading
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
        self.running = [0] * executor.nlanes()   # footprint of the batch each lane runs
        self.skips: dict = {}
        self.log: list = []

    def charged(self, lane) -> int:
        """Device memory of the other lanes: their batches in flight or the
        workspaces they keep, whichever is larger."""
        tot = 0
        for j, b in enumerate(self.running):
            if j == lane:
                continue
            tot += max(b, self.ex.retained(j))
        return tot

    def admit(self, queue: collections.deque, lane: int = 0) -> list:
        chosen, free = [], self.budget - self.charged(lane)
        head_waits = False
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
                if self.skips.get(r.rid, 0) >= self.max_bypass:
                    break                 # bypassed often enough: wait for the head
                head_waits = True
        if head_waits and chosen:
            # a bypass is counted only when requests behind the head go first
            self.skips[queue[0].rid] = self.skips.get(queue[0].rid, 0) + 1
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
                self.in_use -= self.running[lane]
                self.running[lane] = 0
                progressed = True
            while queue:
                lane = self.ex.free_lane()
                if lane is None:
                    break
                chosen = self.admit(queue, lane)
                if not chosen:
                    break
                t = self.ex.now()
                for r in chosen:
                    r.t_start = t
                    r.batch_size = len(chosen)
                fp = sum(self.footprint(r) for r in chosen)
                self.running[lane] = fp
                self.in_use += fp
                self.log.append((t, len(chosen), self.charged(-1)))
                self.ex.launch(lane, chosen)
                progressed = True
            if not progressed:
                self.ex.wait(pending[0].arrival if pending else None)
        return reqs


class GpuExecutor:
    """Lanes = HIP streams with their own context, tree (and workspace),
    buffers and worker thread."""

    def __init__(self, prm=None, k_iter: int = 24, lanes: int = 2, keep_results: bool = False, device=0):
        import torch
        from . import binding as B
        from . import pipeline as P
        self.B, self.P, self.torch = B, P, torch
        self.prm = prm or B.params()
        self.k_iter = k_iter
        self.keep = keep_results
        self.device = device
        self.lanes = []
        for _ in range(lanes):
            st = torch.cuda.Stream(device)
            ctx = B.Context(device, stream=st)
            lane = {"stream": st, "ctx": ctx, "tree": B.Tree(ctx), "reqs": None, "done": threading.Event(),
                    "q": _queue.Queue(), "err": None}
            lane["thread"] = threading.Thread(target=self._worker, args=(lane,), daemon=True)
            lane["thread"].start()
            self.lanes.append(lane)
        self.t0 = time.perf_counter()

    def nlanes(self) -> int:
        return len(self.lanes)

    def retained(self, i) -> int:
        """Workspace bytes lane i keeps: its tree's and, once a batch needed a
        re-run, the auxiliary tree's."""
        tot = 0
        for t in (self.lanes[i]["tree"], getattr(self.lanes[i]["tree"], "_aux", None)):
            ws = None if t is None else t.ws
            tot += 0 if ws is None else int(ws.numel())
        return tot

    def _worker(self, lane):
        torch = self.torch
        torch.cuda.set_device(self.device)
        while True:
            reqs = lane["q"].get()
            if reqs is None:
                return
            try:
                with torch.cuda.stream(lane["stream"]):
                    self._run(lane, reqs)
            except Exception as e:   # reported by completed()
                lane["err"] = e
            lane["done"].set()

    def _run(self, lane, reqs):
        B, P = self.B, self.P
        batch = B.batch_from_sets([r.ps for r in reqs])
        out = P.Outputs(batch.n, batch.nsets)
        P.launch_graph(lane["tree"], batch, self.prm, out, self.k_iter)
        lane["stream"].synchronize()
        P.finish_graph(lane["tree"], batch, self.prm, out, self.k_iter)
        lane["stream"].synchronize()
        sums = out.f.sums.view(-1, 8).cpu().numpy()
        for s, r in enumerate(reqs):
            r.pairs = float(sums[s, 6]) / 2.0
            if self.keep:
                r.result = {k: P.per_set(batch, getattr(out.d, k), s) for k in ("rho", "h", "nngb", "nw")}
                r.result.update({k: P.per_set(batch, getattr(out.f, k), s)
                                 for k in ("ax", "ay", "az", "dudt", "nforce")})

    def close(self):
        for l in self.lanes:
            l["q"].put(None)
        for l in self.lanes:
            l["thread"].join(timeout=30)

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
        l = self.lanes[i]
        l["done"].clear()
        l["reqs"] = reqs
        l["q"].put(reqs)

    def completed(self):
        done = []
        for i, l in enumerate(self.lanes):
            if l["reqs"] and l["done"].is_set():
                if l["err"] is not None:
                    e, l["err"] = l["err"], None
                    raise e
                done.append((i, l["reqs"]))
                l["reqs"] = None
        return done

    def wait(self, next_arrival):
        time.sleep(2e-5)


class FakeExecutor:
    """Simulated clock and service times (for testing the scheduler on a CPU):
    a batch takes `base + per_particle * N` seconds on its lane."""

    def __init__(self, lanes: int = 2, base: float = 1e-3, per_particle: float = 2e-9, retained: int = 0):
        self.lanes = [None] * lanes
        self.base, self.per = base, per_particle
        self.keep = retained     # bytes each lane keeps once it has run a batch
        self.used = [False] * lanes
        self.t = 0.0

    def nlanes(self) -> int:
        return len(self.lanes)

    def retained(self, i) -> int:
        return self.keep if self.used[i] else 0

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
        self.used[i] = True
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
