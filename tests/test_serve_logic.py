"""CPU tests of the served-mode scheduler against a simulated executor:
admission by footprint, head-of-line bypass and its limit, slot reuse,
latency bookkeeping and the p50/p99 summary."""
import numpy as np

from paper_1309_3783_amd.serve import FakeExecutor, Request, Scheduler, summary


class PS:
    def __init__(self, n):
        self.n = n


def fp(r):
    return r.n * 100


def make(ns, arrivals):
    return [Request(i, float(a), PS(n)) for i, (n, a) in enumerate(zip(ns, arrivals))]


def test_all_requests_complete_and_latency_positive():
    rng = np.random.default_rng(0)
    ns = np.round(np.exp(rng.uniform(np.log(1e4), np.log(2e6), 300))).astype(int)
    arr = np.cumsum(rng.exponential(0.002, 300))
    reqs = make(ns, arr)
    sch = Scheduler(FakeExecutor(lanes=2), budget_bytes=400_000_000, footprint=fp)
    out = sch.run(reqs)
    assert all(r.t_done >= r.t_start >= r.arrival for r in out)
    s = summary(out)
    assert s["requests"] == 300 and s["p99_ms"] >= s["p50_ms"] > 0
    # memory in flight never exceeds the budget
    assert max(u for _, _, u in sch.log) <= 400_000_000
    assert sch.in_use == 0


def test_admission_respects_budget_and_batches_arrivals():
    # five small requests arriving together fit in one batch; budget allows 3
    reqs = make([1000] * 5, [0.0] * 5)
    sch = Scheduler(FakeExecutor(lanes=1, base=1.0, per_particle=0.0), budget_bytes=3 * 1000 * 100,
                    footprint=fp)
    sch.run(reqs)
    sizes = [n for _, n, _ in sch.log]
    assert sizes == [3, 2]
    assert reqs[3].t_start == 1.0 and reqs[0].t_done == 1.0


def test_head_of_line_bypass_is_bounded():
    # a big head request that does not fit next to a running one: smaller
    # requests behind it go first, at most max_bypass times
    ns = [600, 900] + [100] * 20
    arr = [0.0, 0.001] + [0.002 + 0.0001 * k for k in range(20)]
    reqs = make(ns, arr)
    sch = Scheduler(FakeExecutor(lanes=2, base=0.01, per_particle=0.0), budget_bytes=1000 * 100,
                    footprint=fp, max_batch=1, max_bypass=3)
    sch.run(reqs)
    big = reqs[1]
    smaller_first = [r for r in reqs[2:] if r.t_start < big.t_start]
    assert 1 <= len(smaller_first) <= 3 + 1
    assert all(r.t_done > 0 for r in reqs)


def test_request_larger_than_budget_is_rejected():
    reqs = make([10_000], [0.0])
    sch = Scheduler(FakeExecutor(), budget_bytes=100, footprint=fp)
    try:
        sch.run(reqs)
    except RuntimeError as e:
        assert "exceeds the whole budget" in str(e)
    else:
        raise AssertionError("expected a rejection")


def test_retained_lane_memory_is_charged():
    # each lane keeps 250 KB once used; with a 600 KB budget and 100 KB
    # requests the first two batches take 4 and 2 requests; after that both
    # lanes retain 250 KB, so a batch may take at most 600 - 250 = 350 KB of
    # the budget (three requests) where it could take four without the charge
    reqs = make([1000] * 12, [0.0] * 12)
    ex = FakeExecutor(lanes=2, base=0.01, per_particle=0.0, retained=250_000)
    sch = Scheduler(ex, budget_bytes=600_000, footprint=fp, max_batch=4)
    sch.run(reqs)
    assert all(r.t_done > 0 for r in reqs)
    assert max(u for _, _, u in sch.log) <= 600_000
    assert [n for _, n, _ in sch.log[:2]] == [4, 2]
    assert len(sch.log) > 2 and max(n for _, n, _ in sch.log[2:]) <= 3


def test_only_real_bypasses_count():
    # A (600) runs on one lane until t = 0.6; B (900) waits from t = 0.001,
    # alone in the queue at first (not a bypass).  Small requests arriving at
    # 0.1, 0.25 and 0.4 (0.1 s each on the other lane) may go before B twice
    # (max_bypass = 2); the third waits for B.
    reqs = make([600, 900, 100, 100, 100], [0.0, 0.001, 0.1, 0.25, 0.4])
    sch = Scheduler(FakeExecutor(lanes=2, base=0.0, per_particle=1e-3), budget_bytes=1000 * 100,
                    footprint=fp, max_batch=1, max_bypass=2)
    sch.run(reqs)
    big = reqs[1]
    assert [r.rid for r in reqs[2:] if r.t_start < big.t_start] == [2, 3]
    assert big.t_start == 0.6 and reqs[4].t_start >= big.t_start
    assert all(r.t_done > 0 for r in reqs)
