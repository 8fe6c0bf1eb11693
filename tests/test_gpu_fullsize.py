"""Full-size parity in the launch configuration the benchmark times (one
slot per seed, default staging, autotuned x-pass schedule), against FP64
oracle values of sampled bins stored in tests/golden/ (written by
tests/golden/make_golden.py, which calls only the oracle):
* 256^3 local NG (f_NL = 5, log-normal A = 1e-2, sigma = 0.5, k* = 20,
  64 log bins), seeds 0 and 3: local256_fp64_oracle.json;
* 512^3 exponential tail (beta = 3, clip 1e-6, A = 5e-3, sigma = 0.3,
  k* = 40, 96 log bins), seed 0, low tail / peak / high tail:
  exptail512_fp64_oracle.json;
* the same two workloads at bins that the path computes on smaller grids
  of the same box (256^3: bins 0, 7, 14 on 32^3, 64^3, 128^3; 512^3: bins
  28, 40 on 256^3, 384^3): local256_small_fp64_oracle.json,
  exptail512_small_fp64_oracle.json.

Bars: FP32 path within 1e-4 relative per sampled bin; FP64 path within
1e-10; mode counts exact.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as f:
        return json.load(f)


def _job_matches(g, job):
    j = g["job"]
    assert (j["N"], j["A"], j["sigma"], j["k_star"], j["map"], j["F_NL"], j["beta"], j["clip"]) == \
        (job.N, job.spectrum.A, job.spectrum.sigma, job.spectrum.k_star, job.ngmap.kind, job.ngmap.F_NL,
         job.ngmap.beta, job.ngmap.clip)


CASES = {
    "local256_fp64_oracle": lambda: W.config_local_ng(256, 64),
    "exptail512_fp64_oracle": lambda: W.config_exptail(512, 96),
    "local256_small_fp64_oracle": lambda: W.config_local_ng(256, 64),
    "exptail512_small_fp64_oracle": lambda: W.config_exptail(512, 96),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("prec,tol", [("f32", 1e-4), ("f64", 1e-10)])
def test_sampled_bins(name, prec, tol):
    g = _golden(name)
    job = CASES[name]()
    _job_matches(g, job)
    seeds = sorted({s["seed"] for s in g["samples"]})
    print(f"full-size {name} {prec}: seeds {seeds}", flush=True)
    with P.Plan(job.N, L=job.L, prec=prec, n_slots=len(job.seeds), autotune=1) as pl:
        for seed in seeds:
            pl.generate_field(seed, seed, job.spectrum, job.ngmap)
        for seed in seeds:
            smp = [s for s in g["samples"] if s["seed"] == seed]
            bins = [s["bin"] for s in smp]
            om, nb = pl.spectrum(seed, job.targets[bins], job.k_lo[bins], job.k_hi[bins])
            for s, o, n in zip(smp, om, nb):
                assert n == s["nmodes"]
                assert s["target"] == job.targets[s["bin"]]
                rel = abs(o - s["omega"]) / abs(s["omega"])
                print(f"  seed {seed} bin {s['bin']} k={s['target']:.2f} rel err {rel:.2e}", flush=True)
                assert rel <= tol
