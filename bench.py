"""Benchmark of the lattice Omega_GW path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-cpu]
                    [--workload local256|exptail512]

Default workload (local256): one step = the whole hot path for one batch:
four realisations (seeds 0..3) of a 256^3 local non-Gaussian field (f_NL = 5,
i.e. F_NL = 3 with the sample <zeta_g^2> subtracted; log-normal A = 1e-2,
sigma = 0.5, k* = 20) are generated on the device, and Omega_GW is computed
in 64 log bins on [k_F, k_Nyquist] for each (7 bins hold no lattice mode and
cost nothing).  exptail512: eight realisations (seeds 0..7) of a 512^3
exponential-tail field (beta = 3, clip 1e-6; A = 5e-3, sigma = 0.3, k* = 40)
in 96 log bins, averaged over the seeds.  Fields and FFTs are FP32
(complex64); maps, lookup tables and shell sums are FP64.  Inputs (plans,
tables) are resident before the timed region.  After the timed region the
FP64 path runs seed 0 (skip with --no-fp64): its speed, the FP32 speedup over
it, and the per-bin FP32 error against it.

Prints one JSON line with the throughput in spectra/s (one spectrum = one
realisation x all its bins), the roofline of the dominant kernel measured
live with HIP events on the plan stream plus the end-to-end fraction of the
two-pass byte model, the timed step's per-bin error against the FP64 oracle
values stored in tests/golden/ (exit status 1 above 1e-4, or above 1e-10
for the FP64 path), and the FP64 oracle timed on the host cores on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch (four realisations per launch, the benchmark's
# configuration and launch mix), averaged over the launches of one spectrum,
# from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes on `bench.py --quick`,
# scaled by a 1 GiB copy (reads x2.0, writes x1.0); valid only for the kernel
# source they were taken on and only for the workload whose launch mix they
# cover (see the summaries in profiles/).
COUNTER_SOURCE_SHA = "defb99cec9076375"
COUNTER_TRAFFIC = {
    "local256": {"xprod": 31462149364.1, "ypass": 49640423669.9, "gen_z": 19115834710.4},
    "exptail512": {"xprod": 54935838040.2, "ypass": 29380982619.7, "gen_z": 11891645119.8},
}


def kernel_source_sha() -> str:
    """Hash of the device code (kernels and the FFT header they include)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("sigw_kernels.hip", "sigw_fft.hpp"):
        with open(os.path.join(ROOT, "paper_2605_27231_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stage_terms(N: int, cb: int, n_alpha: int = 50) -> int:
    """Terms the library stages per gen_z / ypass3 pair with the default plan
    (the largest count whose 2 half spectra per term fit in 16 GiB)."""
    FS = (N // 2 + 1) * N * N
    return max(1, min(n_alpha, (16 << 30) // (2 * FS * cb)))


def lattice_n2(N: int) -> np.ndarray:
    """Which |n|^2 in [0, 3 (N/2)^2] some mode of the N^3 lattice has (|n_c| <= N/2)."""
    h = N // 2
    sq = np.arange(h + 1) ** 2
    two = np.zeros(2 * h * h + 1, bool)
    two[(sq[:, None] + sq[None, :]).ravel()] = True
    three = np.zeros(3 * h * h + 1, bool)
    s2 = np.nonzero(two)[0]
    three[(s2[:, None] + sq[None, :]).ravel()] = True
    return three


def shell_n2_hi(N: int, L: float, k_lo: float, k_hi: float):
    """Largest |n|^2 of a lattice mode in the shell k_lo <= k_F |n| < k_hi
    (None when the shell holds no lattice mode; such a target launches
    nothing); the planes kx <= sqrt of it carry the shell."""
    kF = 2 * math.pi / L
    n2 = np.arange(3 * (N // 2) ** 2 + 1)
    k = kF * np.sqrt(n2)
    sel = n2[(n2 > 0) & (k >= k_lo) & (k < k_hi) & lattice_n2(N)]
    return int(sel[-1]) if len(sel) else None


def support_n2(N: int, L: float, k: float, u_max: float) -> int:
    """Bound on |n|^2 of the modes where phi_a(k_F |n| / k) can be non-zero
    (u below the last grid edge u_max); the same bound the library prunes
    with."""
    kF = 2 * math.pi / L
    r = u_max * k / kF
    r2 = r * r * (1.0 + 1e-12) + 1.0
    n2max = 3 * (N // 2) ** 2
    return n2max if r2 >= n2max else int(r2)


GRID_SIZES = (8, 16, 32, 64, 128, 256, 384, 512)


def target_grid(N: int, L: float, k: float, u_max: float, n2_hi: int) -> int:
    """The lattice a target's convolutions run on, as the library picks it:
    the smallest compiled size M with M > 2 Rc + Kc and M > 2 Kc + 1 (Rc, Kc:
    largest |n_c| of the weighted fields' support and of the shell), if it
    is below N; else N."""
    rc = math.isqrt(support_n2(N, L, k, u_max))
    kc = math.isqrt(n2_hi)
    need = max(2 * rc + kc + 1, 2 * kc + 2)
    if need >= N:
        return N
    return next((m for m in GRID_SIZES if need <= m < N), N)


def algorithmic_bytes(N: int, L: float, cb: int, n_alpha: int, u_max: float, targets, k_lo, k_hi):
    """Compulsory HBM bytes per launch of each hot kernel (each input read
    once, each output written once), averaged over the launches of one
    spectrum: one launch per target with modes and kernel m (gen_z and
    ypass3: one per staged group of st terms), on the lattice the target
    runs on (target_grid).  Only the support of the weighted fields counts:
    rows (kx, ky) with nx^2 + ny^2 <= n2_sup after the z pass, planes
    kx <= kx_sup after the y pass; everything outside is zero and is neither
    read nor written."""
    st_n = stage_terms(N, cb, n_alpha)
    tot = {"gen_z": 0.0, "ypass": 0.0, "xprod": 0.0}
    cnt = {"gen_z": 0, "ypass": 0, "xprod": 0}
    for kt, lo, hi in zip(targets, k_lo, k_hi):
        n2_hi = shell_n2_hi(N, L, lo, hi)
        if n2_hi is None:
            continue                                   # empty shell: no launches
        M = target_grid(N, L, kt, u_max, n2_hi)
        H = M // 2 + 1
        plane = M * M
        # a smaller grid stages more terms in the same buffer
        st = st_n if M == N else min(n_alpha, st_n * ((N // 2 + 1) * N * N) // (H * plane))
        groups = [min(st, n_alpha - a) for a in range(0, n_alpha, st)]
        n2s = min(support_n2(N, L, kt, u_max), 3 * (M // 2) ** 2)
        kxs = min(H - 1, math.isqrt(n2s))
        n_planes = min(H - 1, math.isqrt(n2_hi)) + 1
        ny2 = np.fft.fftfreq(M, 1.0 / M) ** 2
        kx2 = np.arange(kxs + 1)[:, None] ** 2
        rows = int(((kx2 + ny2[None, :]) <= n2s).sum())   # live (kx, ky) rows
        for g in groups:
            # reads Phi_hat on the live rows, writes the (W, Z) pair of each term there
            tot["gen_z"] += (rows * M + 2 * g * rows * M) * cb
            # reads the live rows of the pairs, writes 3 gradient fields per term on kx <= kx_sup
            tot["ypass"] += (2 * g * rows * M + 3 * g * (kxs + 1) * plane) * cb
            cnt["gen_z"] += 1
            cnt["ypass"] += 1
        # reads the 3 n_alpha gradient fields on kx <= kx_sup, writes 6 components on the shell's planes
        tot["xprod"] += (3 * n_alpha * (kxs + 1) * plane + 6 * n_planes * plane) * cb
        cnt["xprod"] += 1
    return {k: (tot[k] / cnt[k] if cnt[k] else 0.0) for k in tot}


def p2_model_bytes(N: int, L: float, cb: int, n_alpha: int, u_max: float, targets, k_lo, k_hi):
    """Bytes per realisation of one spectrum under the two-pass-per-3D-FFT
    model (p = 2: one intermediate HBM round trip per transform; the first
    inverse pass and the last forward pass fused with the weighting and the
    shell sums): per target and kernel m, Phi_hat read once, 3 gradient
    fields per term written and read once, 6 components of Q written and
    read once.  Returns (pruned, dense): pruned counts only the support of
    each target on the grid it runs on (live rows for Phi_hat, planes
    kx <= kx_sup for the fields, the shell's planes for Q), dense counts the
    whole N^3 lattice for every target that holds modes (626 half spectra
    per target at n_alpha = 50)."""
    H_N = N // 2 + 1
    S_N = H_N * N * N * cb
    pruned = dense = 0.0
    for kt, lo, hi in zip(targets, k_lo, k_hi):
        n2_hi = shell_n2_hi(N, L, lo, hi)
        if n2_hi is None:
            continue
        M = target_grid(N, L, kt, u_max, n2_hi)
        H = M // 2 + 1
        plane = M * M
        n2s = min(support_n2(N, L, kt, u_max), 3 * (M // 2) ** 2)
        kxs = min(H - 1, math.isqrt(n2s))
        n_planes = min(H - 1, math.isqrt(n2_hi)) + 1
        ny2 = np.fft.fftfreq(M, 1.0 / M) ** 2
        kx2 = np.arange(kxs + 1)[:, None] ** 2
        rows = int(((kx2 + ny2[None, :]) <= n2s).sum())
        pruned += 2 * (rows * M + 6 * n_alpha * (kxs + 1) * plane + 12 * n_planes * plane) * cb
        dense += 2 * (1 + 6 * n_alpha + 12) * S_N
    return pruned, dense


def load_goldens(workload: str):
    """Stored FP64 oracle values of this workload (tests/golden/*.json,
    written by tests/golden/make_golden.py from the oracle alone):
    {(seed, bin): (omega, nmodes)}."""
    import glob
    out = {}
    prefix = {"local256": "local256", "exptail512": "exptail512"}[workload]
    for path in sorted(glob.glob(os.path.join(ROOT, "tests", "golden", prefix + "*_fp64_oracle.json"))):
        with open(path) as f:
            g = json.load(f)
        for smp in g["samples"]:
            out[(int(smp["seed"]), int(smp["bin"]))] = (float(smp["omega"]), int(smp["nmodes"]))
    return out


def parity_check(per_seed: dict, goldens: dict, tol: float):
    """Per-bin relative error of the timed step's spectra against the stored
    oracle values (every stored bin of every seed the step computed), and
    whether the mode counts are equal."""
    errs, bins, counts_ok = [], [], True
    for (seed, b), (om_ref, nb_ref) in sorted(goldens.items()):
        if seed not in per_seed:
            continue
        om, nb = per_seed[seed]
        if int(nb[b]) != nb_ref:
            counts_ok = False
        errs.append(abs(float(om[b]) - om_ref) / abs(om_ref))
        bins.append([seed, b])
    if not errs:
        return {"max_rel_err": None, "bins": 0, "tol": tol, "ok": True}
    return {"max_rel_err": float(max(errs)), "median_rel_err": float(np.median(errs)), "bins": len(errs),
            "seeds": sorted({s for s, _ in bins}), "nmodes_equal": counts_ok, "tol": tol,
            "ok": bool(max(errs) <= tol and counts_ok),
            "against": "FP64 oracle values stored in tests/golden/ (seed, bin) of this workload"}


def kernel_u_max(N: int, prec: str = "f32") -> float:
    """Last edge of the kernel table's u grid (the support of every phi_a)."""
    import paper_2605_27231_amd as P
    from paper_2605_27231_amd import api
    _, _, edges = api.sigw_kernel_table(P.plan_desc(N, prec=prec), 0)
    return float(edges[-1])


WORKLOADS = {
    "local256": dict(
        job=lambda: W.config_local_ng(256, 64),
        metric="Omega_GW spectra/s (256^3 FP32 fields/FFT, FP64 shell sums)",
        text="local-NG f_NL=5 log-normal (A=1e-2, sigma=0.5, k*=20), 256^3, L=2pi, "
             "64 log bins on [k_F, k_Nyq], seeds 0..3"),
    "exptail512": dict(
        job=lambda: W.config_exptail(512, 96),
        metric="Omega_GW spectra/s (512^3 FP32 fields/FFT, FP64 shell sums)",
        text="exp-tail beta=3 clip 1e-6 log-normal (A=5e-3, sigma=0.3, k*=40), 512^3, L=2pi, "
             "96 log bins on [k_F, k_Nyq], seeds 0..7 averaged"),
}


def run_gpu(args):
    import torch
    import paper_2605_27231_amd as P

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    job = WORKLOADS[args.workload]["job"]()
    seeds = list(job.seeds)
    prec = "f32"
    # all realisations of a step go through each kernel launch together
    # (grid y) when their workspaces fit comfortably (N <= 256: 4 x 18 GB);
    # the autotuner picks the x-pass schedule at creation (outside the timed
    # region)
    batch = len(seeds) if job.N <= 256 else 1
    plan = P.Plan(job.N, L=job.L, prec=prec, n_slots=len(seeds), batch=batch, autotune=1)
    schedule = plan.schedule()[2]
    cb = 8
    per_seed = {}

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def step(lat):
        for g0 in range(0, len(seeds), batch):
            grp = list(range(g0, min(g0 + batch, len(seeds))))
            t0 = time.perf_counter()
            for i in grp:
                plan.generate_field(i, seeds[i], job.spectrum, job.ngmap)
            om_b, nb_b = plan.spectrum_batch(grp, job.targets, job.k_lo, job.k_hi)
            dt = time.perf_counter() - t0
            for j, i in enumerate(grp):
                lat.append(dt)
                per_seed[seeds[i]] = (om_b[j], nb_b[j])
            if job.N > 256:
                say(f"seeds {[seeds[i] for i in grp]}: {dt:.2f} s")
        return om_b[-1], nb_b[-1]

    for i in range(args.warmup):
        tw = time.perf_counter()
        step([])
        say(f"warmup step {i} {time.perf_counter() - tw:.2f}s")
    torch.cuda.synchronize()
    plan.set_timing(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        om, nb = step(lat)
        say(f"timed step {i} done at {time.perf_counter() - t0:.2f}s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_spectra = len(seeds) * args.steps
    value = n_spectra / dt
    n_targets = int((nb > 0).sum())

    times = {k: plan.kernel_time(k) for k in ("gen_z", "ypass", "xprod", "ypass_q", "zbin")}
    plan.set_timing(False)
    u_max = kernel_u_max(job.N, prec)
    ab = {k: int(round(v * batch))
          for k, v in algorithmic_bytes(job.N, job.L, cb, 50, u_max, job.targets, job.k_lo, job.k_hi).items()}
    # dominant kernel: the one with the largest total time in the timed region
    dom = max(("gen_z", "ypass", "xprod"), key=lambda k: times[k][0] * times[k][1])
    ms_d, n_d = times[dom]
    ach = ab[dom] / (ms_d * 1e-3) / 1e9 if ms_d > 0 else 0.0
    kernels = {}
    for k in ("gen_z", "ypass", "xprod"):
        ms, n = times[k]
        gbs = ab[k] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        kernels[k] = {"avg_ms": round(ms, 4), "launches": n, "alg_bytes": ab[k],
                      "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    for k in ("ypass_q", "zbin"):
        ms, n = times[k]
        kernels[k] = {"avg_ms": round(ms, 4), "launches": n}
    lat_ms = np.array(lat) * 1e3
    # end to end: the p = 2 model's bytes of every realisation and target of
    # a step over the measured time per step, and the bytes the kernels of
    # this design actually have to move (their algorithmic bytes x launches)
    p2_pruned, p2_dense = p2_model_bytes(job.N, job.L, cb, 50, u_max, job.targets, job.k_lo, job.k_hi)
    t_step = dt / args.steps
    moved = sum(ab[k] * times[k][1] for k in ("gen_z", "ypass", "xprod")) / args.steps
    e2e = {"p2_bytes_per_step": round(p2_pruned * len(seeds)),
           "p2_frac": round(p2_pruned * len(seeds) / t_step / 1e9 / HBM_PEAK_GBS, 4),
           "p2_dense_bytes_per_step": round(p2_dense * len(seeds)),
           "p2_dense_frac": round(p2_dense * len(seeds) / t_step / 1e9 / HBM_PEAK_GBS, 4),
           "design_bytes_per_step": round(moved),
           "design_GB_s": round(moved / t_step / 1e9, 1),
           "design_frac": round(moved / t_step / 1e9 / HBM_PEAK_GBS, 4),
           "what": "p2: bytes of the two-pass-per-3D-FFT model (Phi_hat once, 3 fields per term and 6 "
                   "components of Q each written and read once, per target and kernel) on each target's "
                   "support and grid (p2) or the whole lattice (p2_dense), over the time per step; design: "
                   "algorithmic bytes of this build's three hot kernels (10 half spectra per term) over the "
                   "time per step"}
    res = {
        "value": value, "dt": dt, "n_targets": n_targets, "omega_seed_last": om.tolist(),
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": (COUNTER_TRAFFIC.get(args.workload, {}).get(dom)
                                 if kernel_source_sha() == COUNTER_SOURCE_SHA else None),
                     "kernel": dom,
                     "alg_bytes_per_launch": ab[dom], "avg_launch_ms": round(ms_d, 4),
                     "launches": n_d, "end_to_end": e2e},
        "kernels": kernels,
        "schedule": schedule,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "what": f"one spectrum (field generation + {len(job.targets)} bins) end to end; "
                               f"the {batch} spectra of a batch complete together"},
        "batch": batch,
        "omega_seed_mean": np.mean([per_seed[s][0] for s in seeds], axis=0).tolist(),
        "targets": job.targets.tolist(),
        "nmodes": nb.tolist(),
    }
    plan.close()
    goldens = load_goldens(args.workload)
    res["parity"] = parity_check(per_seed, goldens, 1e-4)
    if not args.no_fp64:
        pl64 = P.Plan(job.N, L=job.L, prec="f64", n_slots=1, autotune=1)
        say("FP64 path: warm-up spectrum of seed 0")
        pl64.generate_field(0, seeds[0], job.spectrum, job.ngmap)
        pl64.spectrum(0, job.targets, job.k_lo, job.k_hi)   # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pl64.generate_field(0, seeds[0], job.spectrum, job.ngmap)
        om64, nb64 = pl64.spectrum(0, job.targets, job.k_lo, job.k_hi)
        torch.cuda.synchronize()
        d64 = time.perf_counter() - t1
        pl64.close()
        say(f"FP64 path: {d64:.2f} s per spectrum")
        om32 = per_seed[seeds[0]][0]
        ok = nb64 > 0
        rel = np.zeros_like(om64)
        rel[ok] = np.abs(om32[ok] - om64[ok]) / np.abs(om64[ok])
        res["fp64_path"] = {"spectra_per_s": 1.0 / d64, "speedup_fp32_over_fp64": value * d64,
                            "fp32_rel_err_per_bin": {"max": float(rel.max()), "median": float(np.median(rel[ok])),
                                                     "bins": [float(x) for x in rel]},
                            "nmodes_equal": bool(np.array_equal(nb64, per_seed[seeds[0]][1])),
                            "parity": parity_check({seeds[0]: (om64, nb64)}, goldens, 1e-10),
                            "what": f"seed {seeds[0]} only, same bins, FP64 fields/FFTs; one spectrum "
                                    f"timed after a warm-up spectrum, field generation included"}
    return res


def quick_profile(workload: str = "local256"):
    """A short run for hardware-counter passes, in the benchmark's launch
    configuration and launch mix: local256: the four 256^3 fields in one
    batch through every target of the spectrum (one step, so the per-launch
    averages of the counters cover the same launches as the benchmark's);
    exptail512: one 512^3 realisation (the benchmark runs them one at a time)
    through every target; then a plain 1 GiB device copy whose counter
    readings calibrate the byte counters (read 1 GiB, write 1 GiB)."""
    import torch
    import paper_2605_27231_amd as P

    job = WORKLOADS[workload]["job"]()
    b = int(np.argmin(np.abs(job.targets - job.spectrum.k_star * 2 / math.sqrt(3))))
    n = len(job.seeds) if job.N <= 256 else 1
    with P.Plan(job.N, L=job.L, prec="f32", n_slots=n, batch=n, autotune=1) as plan:
        for i, s in enumerate(job.seeds[:n]):
            plan.generate_field(i, s, job.spectrum, job.ngmap)
        om, nb = plan.spectrum_batch(list(range(n)), job.targets, job.k_lo, job.k_hi)
        om, nb = om[0][b:b + 1], nb[0][b:b + 1]
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"quick": True, "target": float(job.targets[b]), "omega": float(om[0]),
                      "nmodes": int(nb[0]), "copy_bytes": 1 << 30}), flush=True)


def stream_probe():
    """The streaming-rate probe (sigw_stream_probe): read, write, copy and the
    2-read : 3-write mix over 1 GiB arrays, fastest of 5 launches each, three
    times; prints one JSON line."""
    import torch
    from paper_2605_27231_amd import api

    names = ("read", "write", "copy", "mix_2r3w")
    res = {n: [] for n in names}
    for _ in range(3):
        for k, n in enumerate(names):
            res[n].append(round(api.sigw_stream_probe(k, 1 << 30, 5), 1))
    torch.cuda.synchronize()
    print(json.dumps({"stream_probe_GB_s": res, "array_bytes": 1 << 30,
                      "what": "fastest of 5 launches per kind, 3 rounds; bytes = arrays touched x 1 GiB"}),
          flush=True)


def cpu_baseline(budget_terms=(1, 6)):
    """The FP64 oracle on a bounded sample: field generation of seed 0, then the
    source convolutions of the sine kernel at the peak target with 1 and 6 of
    the 50 kept terms; the per-term slope and the fixed cost are extrapolated
    linearly to 2 kernels x 50 terms x the non-empty targets of one spectrum."""
    from oracle import decomposition, field, lattice, spectrum

    job = W.config_local_ng(256, 64)
    threads = lattice._WORKERS
    t0 = time.perf_counter()
    tabs = decomposition.tables()
    ph = field.phi_hat(job.N, job.L, 0, job.spectrum, job.ngmap)
    t_gen = time.perf_counter() - t0
    b = int(np.argmin(np.abs(job.targets - job.spectrum.k_star * 2 / math.sqrt(3))))
    k_b = float(job.targets[b])
    ts = []
    for k in budget_terms:
        sub = decomposition.KernelTable(which="s", edges=tabs[0].edges, sigma=tabs[0].sigma[:k],
                                        phi=tabs[0].phi[:, :k], sigma_all=tabs[0].sigma_all,
                                        q_all=tabs[0].q_all)
        t1 = time.perf_counter()
        Q = spectrum.source_qhat(ph, sub, k_b, job.L)
        ts.append(time.perf_counter() - t1)
    t1 = time.perf_counter()
    spectrum.shell_sum(Q, Q, k_b, job.k_lo[b], job.k_hi[b], job.L)
    t_bin = time.perf_counter() - t1
    slope = (ts[1] - ts[0]) / (budget_terms[1] - budget_terms[0])
    fixed = ts[0] - slope * budget_terms[0]
    t_target = 2 * (fixed + 50 * slope) + t_bin
    n_targets = int((spectrum.mode_counts(job.N, job.L, job.k_lo, job.k_hi) > 0).sum())
    t_spec = t_gen + n_targets * t_target
    return {"value": 1.0 / t_spec, "unit": "spectra/s", "cores": threads, "kind": "oracle",
            "sample": (f"256^3 FP64 oracle: seed-0 field generation ({t_gen:.1f} s) + sine-kernel "
                       f"convolutions at k={k_b:.2f} with {budget_terms[0]} and {budget_terms[1]} of 50 "
                       f"terms ({ts[0]:.1f} s, {ts[1]:.1f} s) + one shell sum; extrapolated to "
                       f"2 kernels x 50 terms x {n_targets} targets = {t_spec:.0f} s per spectrum")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path (timed on one seed by default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--quick", action="store_true",
                    help="one field + one target + a 1 GiB copy, for hardware-counter passes")
    ap.add_argument("--workload", default="local256", choices=sorted(WORKLOADS),
                    help="local256 (the headline line) or exptail512")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only the streaming-rate probe (read, write, copy, 2-read:3-write)")
    args = ap.parse_args()
    if args.quick:
        quick_profile(args.workload)
        return
    if args.stream_probe:
        stream_probe()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU mode.  Realisations and "
              "target bins are independent units whose only output is a few KB of shell sums, so "
              "several GPUs would each take a share of them (one process per GPU) and the host "
              "would gather the sums.", file=sys.stderr)
        sys.exit(2)
    g = run_gpu(args)
    wl = WORKLOADS[args.workload]
    job = wl["job"]()
    cpu = None
    if not args.no_cpu and args.workload == "local256":
        print("[bench] oracle CPU baseline sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    line = {
        "metric": wl["metric"],
        "value": round(g["value"], 4),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["dt"] / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["text"], "N": job.N, "bins": len(job.targets),
                   "nonempty_bins": g["n_targets"], "seeds": len(job.seeds),
                   "n_alpha": 50, "n_modes": 200},
        "roofline": g["roofline"],
        "kernels": g["kernels"],
        "xprod_schedule": g["schedule"],
        "latency_ms": g["latency_ms"],
        "cpu_baseline": cpu,
    }
    line["parity"] = g["parity"]
    if "fp64_path" in g:
        line["fp64_path"] = g["fp64_path"]
    if args.workload != "local256":
        line["omega_seed_mean"] = g["omega_seed_mean"]
        line["targets"] = g["targets"]
        line["nmodes"] = g["nmodes"]
    print(json.dumps(line), flush=True)
    # the timed spectra must match the stored oracle values (and the FP64
    # path its own bar): otherwise the throughput above is not a result
    bad = not g["parity"]["ok"] or ("fp64_path" in g and not g["fp64_path"]["parity"]["ok"])
    if bad:
        print("[bench] PARITY FAILURE against the stored oracle values", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
