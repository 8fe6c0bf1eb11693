"""CPU tests of the serving loop's scheduling, with a simulated device and
clock: every request completes, admission respects the HBM budget, idle
plans of other sizes are released for a larger request, requests of one
size overlap on several plans, latencies are accounted from arrival, and a
request that can never fit is refused up front; the caps on requests in
flight and plans per size hold."""
from dataclasses import dataclass

import numpy as np
import pytest

from paper_2605_27231_amd.serve import SpectrumServer, summarize


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 1e-5)


@dataclass
class FakeJob:
    N: int
    seed: int

    @property
    def seeds(self):
        return (self.seed,)


@dataclass
class Req:
    rid: int
    arrival: float
    job: FakeJob


class FakeBackend:
    SERVICE = {32: 0.010, 64: 0.020, 128: 0.050, 384: 0.200}
    FOOT = {32: 1, 64: 2, 128: 4, 384: 10}

    def __init__(self, clock):
        self.clock = clock
        self.created = []
        self.closed = 0

    def footprint(self, N):
        return self.FOOT[N]

    def make_plan(self, N):
        be = self

        class Plan:
            def __init__(self):
                self.job = None
                self.t0 = None
                be.created.append(N)

            def submit(self, job):
                assert self.job is None, "plan submitted twice"
                self.job, self.t0 = job, be.clock()

            def poll(self):
                if be.clock() < self.t0 + be.SERVICE[N]:
                    return None
                job, self.job = self.job, None
                return np.array([job.seed * 1.0, N * 1.0]), np.array([1, 2])

            def close(self):
                be.closed += 1

        return Plan()


def _run(reqs, budget, prewarm=None, **caps):
    clk = SimClock()
    be = FakeBackend(clk)
    caps.setdefault("max_inflight", 100)
    caps.setdefault("max_plans_per_size", 100)
    srv = SpectrumServer(be, budget, clock=clk, idle_wait=clk.wait, prewarm=prewarm, **caps)
    done = srv.serve(reqs)
    return srv, be, done


def test_all_complete_with_correct_results_and_latency():
    reqs = [Req(i, 0.003 * i, FakeJob([32, 64, 128][i % 3], 100 + i)) for i in range(30)]
    srv, be, done = _run(reqs, budget=40)
    assert sorted(d.rid for d in done) == list(range(30))
    for d in done:
        r = reqs[d.rid]
        assert d.omega[0] == r.job.seed and d.omega[1] == r.job.N
        assert d.start >= d.arrival - 1e-12
        assert d.latency >= FakeBackend.SERVICE[d.N] - 1e-9
    s = summarize(done, wall=1.0)
    assert s["completed"] == 30 and s["latency_ms"]["p99"] >= s["latency_ms"]["p50"]


def test_budget_is_never_exceeded_and_requests_queue():
    # budget for exactly one 128 plan: the 128 requests run one after another
    reqs = [Req(i, 0.0, FakeJob(128, i)) for i in range(5)]
    srv, be, done = _run(reqs, budget=4)
    assert srv.peak_used <= 4 and be.created == [128]
    fin = sorted(d.finish for d in done)
    assert all(b - a >= FakeBackend.SERVICE[128] - 1e-9 for a, b in zip(fin, fin[1:]))


def test_same_size_requests_overlap_on_several_plans():
    reqs = [Req(i, 0.0, FakeJob(64, i)) for i in range(4)]
    srv, be, done = _run(reqs, budget=100)
    assert srv.peak_inflight == 4
    assert max(d.finish for d in done) < 2 * FakeBackend.SERVICE[64]


def test_idle_plans_of_other_sizes_are_released():
    # budget 10 holds five 64-plans or one 384-plan
    reqs = [Req(i, 0.0, FakeJob(64, i)) for i in range(5)] + [Req(5, 0.001, FakeJob(384, 5))]
    srv, be, done = _run(reqs, budget=10)
    assert srv.peak_used <= 10
    assert be.created.count(384) == 1 and be.closed >= 5
    d384 = [d for d in done if d.N == 384][0]
    assert d384.start >= FakeBackend.SERVICE[64] - 1e-9     # waited for the 64s to go idle


def test_prewarm_and_oversized_request():
    clk = SimClock()
    be = FakeBackend(clk)
    srv = SpectrumServer(be, 8, clock=clk, idle_wait=clk.wait, prewarm={64: 2, 128: 5})
    assert be.created == [64, 64, 128]          # the rest of the pool would exceed the budget
    with pytest.raises(ValueError):
        srv.serve([Req(0, 0.0, FakeJob(384, 0))])


def test_inflight_and_per_size_caps():
    reqs = [Req(i, 0.0, FakeJob(64, i)) for i in range(10)]
    srv, be, done = _run(reqs, budget=100, max_inflight=8, max_plans_per_size=2)
    assert len(done) == 10 and be.created == [64, 64] and srv.peak_inflight == 2
    mixed = [Req(i, 0.0, FakeJob([32, 64, 128][i % 3], i)) for i in range(9)]
    srv, be, done = _run(mixed, budget=100, max_inflight=3, max_plans_per_size=4)
    assert len(done) == 9 and srv.peak_inflight == 3
    progress = []
    clk = SimClock()
    srv = SpectrumServer(FakeBackend(clk), 100, clock=clk, idle_wait=clk.wait)
    srv.serve([Req(i, 0.0, FakeJob(32, i)) for i in range(500)], progress=lambda d, n: progress.append((d, n)))
    assert progress == [(250, 500), (500, 500)]
