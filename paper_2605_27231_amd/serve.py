"""Continuous-batching spectrum server.

Requests (a lattice size, a Gaussian spectrum, a map, a seed and a few
target shells) arrive over time.  Each request runs on a plan of its size;
plans live in per-size pools, each plan on its own HIP stream, so work of
several requests overlaps on the device.  A request is admitted as soon as
a plan of its size is idle, or a new plan fits the HBM budget (idle plans
of other sizes are released first if needed); otherwise it waits.  Every
result comes back through the plan's asynchronous spectrum entry points, and
the latency from arrival to result is recorded.

    python -m paper_2605_27231_amd.serve --requests 300 --rate 50

The scheduling logic is independent of the device: a backend supplies plan
footprints and plan objects (submit / poll / close), so the same loop runs
against the HIP library or, in tests, against a simulated device.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass
class Served:
    rid: int
    N: int
    arrival: float
    start: float
    finish: float
    omega: np.ndarray
    nmodes: np.ndarray

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class GpuBackend:
    """Plans of the HIP library, one stream each.  The largest lattices use
    fewer terms per workspace pass (alpha_chunk) so that several plans stay
    resident: at 384^3, 25 terms per pass cost 3% more time per request than
    all 50 (54 GB plans) and 10 terms cost 15%; at 256^3 and below every term
    shares one pass (measured with --service-times)."""

    def __init__(self, prec: str = "f32", chunk_for=None):
        self.prec = prec
        self.chunk_for = chunk_for or (lambda N: 25 if N >= 384 else 0)

    def _desc(self, N):
        from .api import plan_desc
        return plan_desc(N, prec=self.prec, alpha_chunk=self.chunk_for(N), autotune=1)

    def footprint(self, N: int) -> int:
        from .api import sigw_plan_footprint
        return sigw_plan_footprint(self._desc(N))

    def make_plan(self, N: int):
        return _GpuPlan(N, self.prec, self.chunk_for(N))


class _GpuPlan:
    def __init__(self, N, prec, chunk):
        import torch
        from .api import Plan
        self.stream = torch.cuda.Stream()
        self.plan = Plan(N, prec=prec, n_slots=1, alpha_chunk=chunk, stream=self.stream, autotune=1)

    def submit(self, job):
        self.plan.generate_field(0, int(job.seeds[0]), job.spectrum, job.ngmap)
        self.plan.spectrum_enqueue(0, job.targets, job.k_lo, job.k_hi)

    def poll(self):
        return self.plan.spectrum_poll()

    def close(self):
        self.plan.close()


class SpectrumServer:
    """max_inflight bounds the requests on the device at once and
    max_plans_per_size the plans kept per lattice size: the device has a few
    hardware queues, so more concurrent streams add memory and host work
    (plan creation) without adding throughput."""

    def __init__(self, backend, budget_bytes: int, clock: Callable[[], float] = time.perf_counter,
                 idle_wait: Callable[[float], None] = time.sleep, prewarm: Optional[Dict[int, int]] = None,
                 max_inflight: int = 8, max_plans_per_size: int = 4):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.max_plans_per_size = int(max_plans_per_size)
        self.clock = clock
        self.idle_wait = idle_wait
        self.used = 0
        self.free: Dict[int, List] = {}
        self.idle_since: Dict[int, float] = {}
        self.n_plans: Dict[int, int] = {}
        self.peak_used = 0
        self.peak_inflight = 0
        for N, n in (prewarm or {}).items():
            for _ in range(min(n, self.max_plans_per_size)):
                if not self._create(N):
                    break

    # -- pool management ---------------------------------------------------------
    def _create(self, N: int) -> bool:
        fp = self.backend.footprint(N)
        if self.used + fp > self.budget:
            return False
        plan = self.backend.make_plan(N)
        plan._fp = fp
        plan._N = N
        self.used += fp
        self.peak_used = max(self.peak_used, self.used)
        self.n_plans[N] = self.n_plans.get(N, 0) + 1
        self.free.setdefault(N, []).append(plan)
        self.idle_since[id(plan)] = self.clock()
        return True

    def _release_idle(self, need: int, keep_N: int) -> None:
        """Free idle plans of other sizes, longest idle first, until `need`
        more bytes fit."""
        cands = [(self.idle_since.get(id(p), 0.0), N, p) for N, ps in self.free.items() if N != keep_N
                 for p in ps]
        cands.sort(key=lambda c: c[0])
        for _, N, p in cands:
            if self.used + need <= self.budget:
                break
            self.free[N].remove(p)
            self.used -= p._fp
            self.n_plans[N] -= 1
            p.close()

    def _acquire(self, N: int):
        ps = self.free.get(N)
        if ps:
            return ps.pop()
        if self.n_plans.get(N, 0) >= self.max_plans_per_size:
            return None
        fp = self.backend.footprint(N)
        if fp > self.budget:
            raise ValueError(f"a plan for N={N} needs {fp} bytes, more than the whole budget")
        if self.used + fp > self.budget:
            self._release_idle(fp, N)
        if self._create(N):
            return self.free[N].pop()
        return None

    def close(self):
        for ps in self.free.values():
            for p in ps:
                p.close()
        self.free.clear()
        self.used = 0

    # -- the loop ----------------------------------------------------------------
    def serve(self, requests, progress: Optional[Callable[[int, int], None]] = None) -> List[Served]:
        """requests: objects with rid, arrival (seconds after start) and job,
        in arrival order.  Returns one Served per request, in finish order.
        progress(done, total) is called after every 250th completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if self.backend.footprint(r.job.N) > self.budget:
                raise ValueError(f"request {r.rid}: N={r.job.N} does not fit the budget")
        t0 = self.clock()
        waiting = deque()
        busy = {}
        done: List[Served] = []
        i = 0
        while len(done) < len(reqs):
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                waiting.append(reqs[i])
                i += 1
            admitted = False
            # first fit over the waiting requests, oldest first
            for req in list(waiting):
                if len(busy) >= self.max_inflight:
                    break
                plan = self._acquire(req.job.N)
                if plan is None:
                    continue
                waiting.remove(req)
                plan.submit(req.job)
                busy[id(plan)] = (plan, req, self.clock() - t0)
                admitted = True
            self.peak_inflight = max(self.peak_inflight, len(busy))
            finished = False
            for key, (plan, req, t_start) in list(busy.items()):
                res = plan.poll()
                if res is None:
                    continue
                t_fin = self.clock() - t0
                om, nb = res
                done.append(Served(req.rid, req.job.N, req.arrival, t_start, t_fin, np.asarray(om),
                                   np.asarray(nb)))
                del busy[key]
                self.free.setdefault(plan._N, []).append(plan)
                self.idle_since[id(plan)] = self.clock()
                finished = True
                if progress is not None and len(done) % 250 == 0:
                    progress(len(done), len(reqs))
            if not admitted and not finished:
                # nothing moved: wait a little, never past the next arrival
                nxt = reqs[i].arrival - (self.clock() - t0) if i < len(reqs) else math.inf
                self.idle_wait(max(0.0, min(2e-4, nxt)))
        return done


def summarize(done: List[Served], wall: float) -> dict:
    lat = np.array([d.latency for d in done]) * 1e3
    sizes = {}
    for d in done:
        sizes.setdefault(d.N, []).append(d.latency * 1e3)
    return {
        "completed": len(done),
        "wall_s": wall,
        "req_per_s": len(done) / wall if wall > 0 else float("nan"),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "max": float(lat.max())},
        "by_N": {str(N): {"n": len(v), "p50_ms": float(np.percentile(v, 50)),
                          "p99_ms": float(np.percentile(v, 99))} for N, v in sorted(sizes.items())},
    }


def service_times(sizes, chunks, prec: str = "f32", reps: int = 3, n_targets: int = 4) -> dict:
    """Device time of one request of each lattice size run alone (field
    generation + n_targets thin shells around the peak), for each alpha_chunk
    in chunks: the per-size service times that bound the served rate.  The
    capacity at the stream's N mix is 1 / sum_N weight_N t_N."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    import workloads as W
    from .api import Plan, plan_desc, sigw_plan_footprint

    out = {}
    for N in sizes:
        req = next(r for r in W.request_stream(400, 50.0, sizes=sizes) if r.job.N == N)
        job = req.job
        for ch in chunks:
            fp = sigw_plan_footprint(plan_desc(N, prec=prec, alpha_chunk=ch))
            with Plan(N, prec=prec, alpha_chunk=ch, autotune=1) as pl:
                ts = []
                for r in range(reps + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    pl.generate_field(0, int(job.seeds[0]), job.spectrum, job.ngmap)
                    pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
                    torch.cuda.synchronize()
                    if r:
                        ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            out[f"{N}/chunk{ch}"] = {"N": N, "alpha_chunk": ch, "ms_per_request": round(t * 1e3, 3),
                                     "ms_per_target": round(t * 1e3 / n_targets, 3), "plan_GB": round(fp / 1e9, 2)}
            print(f"[service] N={N} alpha_chunk={ch}: {t * 1e3:.2f} ms per request ({fp / 1e9:.1f} GB plan)",
                  file=sys.stderr, flush=True)
    return out


def main():
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--prec", default="f32")
    ap.add_argument("--sizes", default="64,128,256,384")
    ap.add_argument("--max-inflight", type=int, default=8)
    ap.add_argument("--plans-per-size", type=int, default=4)
    ap.add_argument("--service-times", action="store_true",
                    help="only time one request of each size alone, at alpha_chunk 0 / 10 / 25")
    args = ap.parse_args()
    sizes = tuple(int(s) for s in args.sizes.split(","))
    weights = {64: 0.4, 128: 0.3, 256: 0.2, 384: 0.1}
    w = np.array([weights.get(n, 1.0) for n in sizes])
    if args.service_times:
        st = service_times(sizes, (0, 10, 25), args.prec)
        best = {N: min(v["ms_per_request"] for v in st.values() if v["N"] == N) for N in sizes}
        mean = float(sum(wt * best[N] for N, wt in zip(sizes, w / w.sum())))
        print(json.dumps({"service": st, "best_ms_per_request": best, "mean_ms_at_mix": round(mean, 3),
                          "capacity_req_per_s": round(1e3 / mean, 2),
                          "what": "one request (field + 4 thin shells) alone per size; capacity = 1 / mean "
                                  "service time at the stream's N mix with the fastest chunking per size"}),
              flush=True)
        return
    reqs = W.request_stream(args.requests, args.rate, sizes=sizes, weights=tuple(w / w.sum()))
    backend = GpuBackend(args.prec)
    prewarm = {64: 4, 128: 4, 256: 3, 384: 2}
    server = SpectrumServer(backend, int(args.budget_gb * 1e9),
                            prewarm={n: min(prewarm.get(n, 1), args.plans_per_size) for n in sizes},
                            max_inflight=args.max_inflight, max_plans_per_size=args.plans_per_size)
    # warm every pooled plan once so that first-use costs stay out of the timing
    warm = [W.Request(rid=-1 - k, arrival=0.0, job=r.job) for k, r in enumerate(reqs[:8])]
    server.serve(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = server.serve(reqs, progress=lambda d, n: print(f"[serve] {d}/{n} done at "
                                                        f"{time.perf_counter() - t0:.1f} s",
                                                        file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    out = summarize(done, wall)
    out.update({"rate": args.rate, "sizes": sizes, "prec": args.prec, "budget_gb": args.budget_gb,
                "max_inflight": args.max_inflight, "plans_per_size": args.plans_per_size,
                "peak_inflight": server.peak_inflight, "plans": server.n_plans,
                "targets_per_request": int(len(reqs[0].job.targets))})
    print(json.dumps(out), flush=True)
    server.close()


if __name__ == "__main__":
    main()
