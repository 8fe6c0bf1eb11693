"""Full-size parity against FP64 oracle values stored in tests/golden/
(written by tests/golden/make_golden.py, which calls only the oracle):

* the benchmark's own launch configuration at 256^3 (local NG, f_NL = 5,
  log-normal A = 1e-2, sigma = 0.5, k* = 20, 64 log bins): one plan with
  four slots, the four realisations (seeds 0..3) of every launch together
  (batch 4), autotuned x-pass schedule, one batched spectrum over all 64
  bins, compared with every stored bin: seed 0 at each of the 57 bins that
  hold modes (local256_seed0_all_fp64_oracle.json), seeds 1..3 at 8 bins
  each (local256_seeds123_fp64_oracle.json), and the earlier samples
  (local256_fp64_oracle.json, local256_small_fp64_oracle.json); each
  realisation of the batch also equals, bit for bit, itself computed alone
  (batch 1);
* the FP64 path on seed 0 at every stored bin;
* 512^3 exponential tail (beta = 3, clip 1e-6, A = 5e-3, sigma = 0.3,
  k* = 40, 96 log bins), seed 0, one realisation per launch as the
  benchmark runs it: low tail / peak / high tail
  (exptail512_fp64_oracle.json) and bins 28, 40, which run on 256^3 and
  384^3 grids (exptail512_small_fp64_oracle.json).

Bars: FP32 path within 1e-4 relative per stored bin; FP64 path within
1e-10; mode counts exact.
"""
import glob
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2605_27231_amd")

HERE = os.path.dirname(os.path.abspath(__file__))


def _goldens(prefix):
    """{(seed, bin): (omega, nmodes)} over every stored file of a workload."""
    out = {}
    for path in sorted(glob.glob(os.path.join(HERE, "golden", prefix + "*_fp64_oracle.json"))):
        with open(path) as f:
            g = json.load(f)
        for s in g["samples"]:
            out[(int(s["seed"]), int(s["bin"]))] = (float(s["omega"]), int(s["nmodes"]), g["job"], s)
    return out


def _job_matches(j, job):
    assert (j["N"], j["A"], j["sigma"], j["k_star"], j["map"], j["F_NL"], j["beta"], j["clip"]) == \
        (job.N, job.spectrum.A, job.spectrum.sigma, job.spectrum.k_star, job.ngmap.kind, job.ngmap.F_NL,
         job.ngmap.beta, job.ngmap.clip)


def _compare(gold, job, seed, om, nb, tol, what):
    worst = 0.0
    n = 0
    for (s, b), (ref, nref, j, smp) in sorted(gold.items()):
        if s != seed:
            continue
        _job_matches(j, job)
        assert smp["target"] == job.targets[b]
        assert nb[b] == nref, (what, seed, b, nb[b], nref)
        rel = abs(om[b] - ref) / abs(ref)
        worst = max(worst, rel)
        n += 1
        assert rel <= tol, (what, seed, b, rel)
    print(f"  {what} seed {seed}: {n} stored bins, max rel err {worst:.2e}", flush=True)
    return n


def test_local256_benchmark_configuration():
    gold = _goldens("local256")
    job = W.config_local_ng(256, 64)
    seeds = list(job.seeds)
    print(f"full-size local256 f32 batch 4 over seeds {seeds}: {len(gold)} stored bins", flush=True)
    with P.Plan(job.N, L=job.L, prec="f32", n_slots=len(seeds), batch=len(seeds), autotune=1) as pl:
        for i, s in enumerate(seeds):
            pl.generate_field(i, s, job.spectrum, job.ngmap)
        om4, nb4 = pl.spectrum_batch(list(range(len(seeds))), job.targets, job.k_lo, job.k_hi)
    n = sum(_compare(gold, job, s, om4[i], nb4[i], 1e-4, "f32 batch 4") for i, s in enumerate(seeds))
    assert n >= len(gold)
    # every realisation of the batch equals itself alone (batch 1), bit for bit
    print("  the same seeds one at a time (batch 1)", flush=True)
    with P.Plan(job.N, L=job.L, prec="f32", n_slots=1, autotune=1) as pl:
        for i, s in enumerate(seeds):
            pl.generate_field(0, s, job.spectrum, job.ngmap)
            om1, nb1 = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
            np.testing.assert_array_equal(om1, om4[i])
            np.testing.assert_array_equal(nb1, nb4[i])


def test_local256_fp64_path():
    gold = _goldens("local256")
    job = W.config_local_ng(256, 64)
    print("full-size local256 f64 seed 0", flush=True)
    with P.Plan(job.N, L=job.L, prec="f64", n_slots=1, autotune=1) as pl:
        pl.generate_field(0, 0, job.spectrum, job.ngmap)
        om, nb = pl.spectrum(0, job.targets, job.k_lo, job.k_hi)
    assert _compare(gold, job, 0, om, nb, 1e-10, "f64") > 0


@pytest.mark.parametrize("prec,tol", [("f32", 1e-4), ("f64", 1e-10)])
def test_exptail512_sampled_bins(prec, tol):
    gold = _goldens("exptail512")
    job = W.config_exptail(512, 96)
    bins = sorted({b for (_, b) in gold})
    print(f"full-size exptail512 {prec} seed 0 bins {bins}", flush=True)
    with P.Plan(job.N, L=job.L, prec=prec, n_slots=1, autotune=1) as pl:
        pl.generate_field(0, 0, job.spectrum, job.ngmap)
        om_b, nb_b = pl.spectrum(0, job.targets[bins], job.k_lo[bins], job.k_hi[bins])
    om = np.zeros(len(job.targets))
    nb = np.zeros(len(job.targets), dtype=np.int64)
    om[bins], nb[bins] = om_b, nb_b
    assert _compare(gold, job, 0, om, nb, tol, prec) == len(bins)
