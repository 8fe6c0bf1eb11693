"""Write FP64 oracle values for the full-size parity tests (sampled bins).

    python tests/golden/make_golden.py [name ...]

Calls only the oracle and the workload recipes; the GPU path never writes
anything here.  Each fixture records the workload, the sampled targets and
the oracle's Omega and mode counts per target.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import decomposition, field, spectrum  # noqa: E402


def _job_dict(job):
    return {"N": job.N, "L": job.L, "A": job.spectrum.A, "sigma": job.spectrum.sigma,
            "k_star": job.spectrum.k_star, "map": job.ngmap.kind, "F_NL": job.ngmap.F_NL,
            "G_NL": job.ngmap.G_NL, "beta": job.ngmap.beta, "clip": job.ngmap.clip}


def _write(out, name):
    tmp = os.path.join(HERE, name + ".json.tmp")
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1)
    os.replace(tmp, os.path.join(HERE, name + ".json"))


def nonempty_bins(job):
    """Bins whose shell holds at least one lattice mode (oracle mode count)."""
    nb = spectrum.mode_counts(job.N, job.L, job.k_lo, job.k_hi)
    return [int(b) for b in np.nonzero(nb > 0)[0]]


def sampled(job, seeds_bins, name, note):
    tabs = decomposition.tables()
    out = {"name": name, "note": note, "job": _job_dict(job), "samples": [],
           "generated_by": "python tests/golden/make_golden.py " + name}
    for seed, bins in seeds_bins:
        t0 = time.time()
        ph = field.phi_hat(job.N, job.L, seed, job.spectrum, job.ngmap)
        for b in bins:
            om, nb = spectrum.omega_target(ph, tabs[0], tabs[1], job.targets[b], job.k_lo[b],
                                           job.k_hi[b], job.L)
            out["samples"].append({"seed": seed, "bin": int(b), "target": float(job.targets[b]),
                                   "k_lo": float(job.k_lo[b]), "k_hi": float(job.k_hi[b]),
                                   "omega": float(om), "nmodes": int(nb)})
            print(name, seed, b, om, nb, f"{time.time() - t0:.0f}s", flush=True)
            _write(out, name)      # after every sample, so that a long run keeps what it has
    _write(out, name)


def ensemble_sampled(jobs, bins, name, note):
    """Sampled bins of several realisations, each with its own parameters."""
    tabs = decomposition.tables()
    out = {"name": name, "note": note, "jobs": [_job_dict(j) | {"seed": int(j.seeds[0])} for j in jobs],
           "samples": [], "generated_by": "python tests/golden/make_golden.py " + name}
    for r, job in enumerate(jobs):
        t0 = time.time()
        ph = field.phi_hat(job.N, job.L, job.seeds[0], job.spectrum, job.ngmap)
        for b in bins:
            om, nb = spectrum.omega_target(ph, tabs[0], tabs[1], job.targets[b], job.k_lo[b], job.k_hi[b], job.L)
            out["samples"].append({"realisation": r, "bin": int(b), "target": float(job.targets[b]),
                                   "omega": float(om), "nmodes": int(nb)})
            print(name, r, b, om, nb, f"{time.time() - t0:.0f}s", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)


FIXTURES = {
    # 256^3 local NG, seed 0 at every bin that holds modes (57 of 64), and
    # seeds 1..3 at 8 bins each spanning the smaller grids, the rise, the
    # peak, the tail and the Nyquist corner: the whole spectrum the
    # benchmark computes, in its batch-of-four launch configuration
    "local256_seeds123_fp64_oracle": lambda: sampled(
        W.config_local_ng(256, 64), [(s, [0, 9, 16, 24, 33, 44, 53, 63]) for s in (1, 2, 3)],
        "local256_seeds123_fp64_oracle",
        "256^3 local NG f_NL=5 (F_NL=3), A=1e-2, sigma=0.5, k*=20, 64 log bins, seeds 1..3 x 8 bins; "
        "FP64 oracle"),
    "local256_seed0_all_fp64_oracle": lambda: sampled(
        W.config_local_ng(256, 64), [(0, nonempty_bins(W.config_local_ng(256, 64)))],
        "local256_seed0_all_fp64_oracle",
        "256^3 local NG f_NL=5 (F_NL=3), A=1e-2, sigma=0.5, k*=20, 64 log bins, seed 0, every "
        "non-empty bin; FP64 oracle"),
    # 256^3 local NG (f_NL = 5), 64 log bins, seeds 0..3: low tail, rise, peak, high tail
    "local256_fp64_oracle": lambda: sampled(
        W.config_local_ng(256, 64), [(0, [20, 33, 44, 60]), (3, [44])], "local256_fp64_oracle",
        "256^3 local NG f_NL=5 (F_NL=3), A=1e-2, sigma=0.5, k*=20, 64 log bins; FP64 oracle"),
    # 512^3 exponential tail (beta = 3), 96 log bins, seed 0: low tail, peak, high tail
    "exptail512_fp64_oracle": lambda: sampled(
        W.config_exptail(512, 96), [(0, [44, 66, 80])], "exptail512_fp64_oracle",
        "512^3 exp-tail beta=3 clip 1e-6, A=5e-3, sigma=0.3, k*=40, 96 log bins; FP64 oracle"),
    # the same two workloads at targets that the hot path computes on smaller
    # grids of the same box (32^3, 64^3, 128^3 for the 256^3 lattice; 256^3
    # and 384^3 for the 512^3 one)
    "local256_small_fp64_oracle": lambda: sampled(
        W.config_local_ng(256, 64), [(0, [0, 7, 14])], "local256_small_fp64_oracle",
        "256^3 local NG f_NL=5 (F_NL=3), A=1e-2, sigma=0.5, k*=20, 64 log bins, bins 0/7/14; FP64 oracle"),
    "exptail512_small_fp64_oracle": lambda: sampled(
        W.config_exptail(512, 96), [(0, [28, 40])], "exptail512_small_fp64_oracle",
        "512^3 exp-tail beta=3 clip 1e-6, A=5e-3, sigma=0.3, k*=40, 96 log bins, bins 28/40; FP64 oracle"),
    # the first four realisations of the 128^3 ensemble (parameters drawn per realisation), 32 log bins
    "ensemble128_fp64_oracle": lambda: ensemble_sampled(
        W.config_ensemble(128, 4, 32), [10, 18, 24], "ensemble128_fp64_oracle",
        "128^3 local NG, per-realisation f_NL, sigma, k* (PCG64 seed 2605), 32 log bins, "
        "realisations 0..3; FP64 oracle"),
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(FIXTURES)
    for n in names:
        FIXTURES[n]()
