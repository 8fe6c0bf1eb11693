"""The stored FP64 oracle values under tests/golden/ (CPU).

The full-size GPU parity tests and the benchmark's self-check compare with
these files, so their metadata is checked here against the workload recipes
and the oracle, independently of the values' own generation:

* each file names the generator script and fixture that wrote it, and its
  recorded workload is the recipe's (lattice, box, spectrum, map);
* every sample's target and shell edges are the recipe's values at that
  bin, and its mode count is the oracle's count of lattice modes in the
  shell;
* a (seed, bin) stored in two files carries the same Omega: the oracle is
  deterministic across separate runs;
* the 256^3 seed-0 file holds every bin that has modes.
"""
import glob
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import spectrum

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _recipe(name):
    if name.startswith("local256"):
        return W.config_local_ng(256, 64)
    if name.startswith("exptail512"):
        return W.config_exptail(512, 96)
    raise KeyError(name)


def _job_dict(job):
    return {"N": job.N, "L": job.L, "A": job.spectrum.A, "sigma": job.spectrum.sigma,
            "k_star": job.spectrum.k_star, "map": job.ngmap.kind, "F_NL": job.ngmap.F_NL,
            "G_NL": job.ngmap.G_NL, "beta": job.ngmap.beta, "clip": job.ngmap.clip}


def _files():
    return sorted(p for p in glob.glob(os.path.join(GOLDEN, "*_fp64_oracle.json"))
                  if not os.path.basename(p).startswith("ensemble"))


def _load(path):
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("path", _files(), ids=lambda p: os.path.basename(p))
def test_golden_metadata_and_mode_counts(path):
    g = _load(path)
    name = os.path.basename(path)[:-len(".json")]
    assert g["name"] == name
    assert g["generated_by"] == "python tests/golden/make_golden.py " + name
    job = _recipe(name)
    assert g["job"] == _job_dict(job)
    samples = g["samples"]
    assert samples
    bins = sorted({int(s["bin"]) for s in samples})
    ref = dict(zip(bins, spectrum.mode_counts(job.N, job.L, job.k_lo[bins], job.k_hi[bins])))
    for s in samples:
        b = int(s["bin"])
        assert s["target"] == float(job.targets[b])
        assert s["k_lo"] == float(job.k_lo[b]) and s["k_hi"] == float(job.k_hi[b])
        assert s["nmodes"] == ref[b] > 0
        assert math.isfinite(s["omega"]) and s["omega"] > 0.0


def test_golden_values_agree_across_files():
    seen = {}
    n_shared = 0
    for path in _files():
        g = _load(path)
        for s in g["samples"]:
            key = (g["job"]["N"], g["job"]["map"], int(s["seed"]), int(s["bin"]))
            if key in seen:
                n_shared += 1
                assert s["nmodes"] == seen[key][1]
                assert abs(s["omega"] - seen[key][0]) <= 1e-12 * abs(seen[key][0]), key
            else:
                seen[key] = (s["omega"], s["nmodes"])
    assert n_shared > 0


def test_seed0_file_covers_every_bin_with_modes():
    job = W.config_local_ng(256, 64)
    g = _load(os.path.join(GOLDEN, "local256_seed0_all_fp64_oracle.json"))
    counts = spectrum.mode_counts(job.N, job.L, job.k_lo, job.k_hi)
    want = [int(b) for b in np.nonzero(counts > 0)[0]]
    assert len(want) == 57
    assert sorted(int(s["bin"]) for s in g["samples"] if s["seed"] == 0) == want
