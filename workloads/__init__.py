"""Seeded synthetic input recipes shared by the oracle and the GPU path.

This module holds only the *inputs* of the computation: lattice sizes, box
length, log-normal power-spectrum parameters, the non-Gaussian map parameters,
bin edges and target wavenumbers, seeds, and the parameter draws of the
ensemble and served-stream workloads.  It holds none of the method's
arithmetic (no kernels, no transforms, no spectra), so that the oracle and the
HIP path can both take their inputs from here without sharing method code.

All boxes use L = 2*pi, so the fundamental mode k_F = 2*pi/L = 1 equals the
infrared unit k_IR in which the peak positions are quoted (a box of 2*pi*32/k_IR
would put the Nyquist frequency below the peak and leave the lattice empty).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi

MAP_GAUSS = "gauss"
MAP_LOCAL = "local"
MAP_EXPTAIL = "exptail"
MAP_NONLOCAL = "nonlocal"


@dataclass(frozen=True)
class Lognormal:
    """Log-normal peak of the dimensionless curvature spectrum, Eq. (lognormal):
    Delta^2(k) = A / sqrt(2 pi sigma^2) * exp(-ln^2(k/k_star) / (2 sigma^2))."""
    A: float
    sigma: float
    k_star: float


@dataclass(frozen=True)
class NGMap:
    """Non-Gaussian map applied to the Gaussian field zeta_g.

    kind = "gauss":   zeta = zeta_g
    kind = "local":   zeta = zeta_g + F_NL (zeta_g^2 - <zeta_g^2>) + G_NL zeta_g^3
                      (Sec. VI B; <zeta_g^2> is the FP64 sample mean over the
                      lattice, which only moves the k = 0 mode)
    kind = "exptail": zeta = -ln(max(1 - beta zeta_g, clip)) / beta
    kind = "nonlocal": zeta = zeta_g + (alpha_NL / k_NL^2) lap(zeta_g^2)
                              + (beta_NL / k_NL^2) zeta_g lap(zeta_g)
                      (Eq. nonlocal; k_NL is the peak scale k* of the spectrum)
    """
    kind: str = MAP_GAUSS
    F_NL: float = 0.0
    G_NL: float = 0.0
    beta: float = 0.0
    clip: float = 1e-6
    alpha_NL: float = 0.0
    beta_NL: float = 0.0
    k_NL: float = 0.0


@dataclass(frozen=True)
class Decomposition:
    """Meta-parameters of the separable kernel decomposition (Sec. V).  The
    paper quotes u_p = 1 in two figure captions and 0.8 in the text, and 200
    intervals in most places but 100 once; the majority values are used."""
    n_modes: int = 200
    n_alpha: int = 50
    u_min: float = 1e-3
    u_max: float = 15.0
    u_p: float = 1.0
    sigma_p: float = 0.5
    A_p: float = 10.0


@dataclass
class Job:
    """One spectrum request: a lattice, a Gaussian spectrum, a map, bins, seeds."""
    N: int
    L: float
    spectrum: Lognormal
    ngmap: NGMap
    k_lo: np.ndarray           # n_k shell lower edges (inclusive)
    k_hi: np.ndarray           # n_k shell upper edges (exclusive)
    targets: np.ndarray        # n_k target wavenumbers, one per shell
    seeds: Tuple[int, ...] = (0,)
    name: str = ""


def fundamental(L: float) -> float:
    return TWO_PI / L


def linear_bins(N: int, L: float, n_bins: int) -> Tuple[np.ndarray, np.ndarray]:
    """Linear bins of width k_F: centres b*k_F (b = 1..n_bins), edges (b -+ 1/2) k_F."""
    kf = fundamental(L)
    b = np.arange(1, n_bins + 1, dtype=np.float64)
    edges = (np.arange(0, n_bins + 1, dtype=np.float64) + 0.5) * kf
    return edges, b * kf


def log_bins(N: int, L: float, n_bins: int) -> Tuple[np.ndarray, np.ndarray]:
    """Log-spaced edges on [k_F, k_Nyquist] with geometric centres."""
    kf = fundamental(L)
    knyq = kf * (N // 2)
    edges = kf * (knyq / kf) ** (np.arange(n_bins + 1, dtype=np.float64) / n_bins)
    edges[0] = kf
    edges[-1] = knyq
    targets = np.sqrt(edges[:-1] * edges[1:])
    return edges, targets


def thin_shells(targets: np.ndarray, L: float) -> Tuple[np.ndarray, np.ndarray]:
    """Thin shells k_b -+ pi/L, one fundamental mode wide (Sec. IV shell
    estimator).  Returns the [lo, hi) edges of each shell."""
    half = 0.5 * fundamental(L)
    t = np.asarray(targets, dtype=np.float64)
    return t - half, t + half


def shells_from_edges(edges: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Contiguous bins [e_{b-1}, e_b) as per-target shells."""
    e = np.asarray(edges, dtype=np.float64)
    return e[:-1].copy(), e[1:].copy()


# --------------------------------------------------------------------------
# The five workload descriptions.
# --------------------------------------------------------------------------

def config_plain_fp64(N: int = 32) -> Job:
    """Gaussian field on 32^3, A=1e-2, sigma=0.5, k*=6, seed 0, 16 linear bins."""
    L = TWO_PI
    e, t = linear_bins(N, L, N // 2)
    lo, hi = shells_from_edges(e)
    return Job(N=N, L=L, spectrum=Lognormal(1e-2, 0.5, 6.0), ngmap=NGMap(MAP_GAUSS),
               k_lo=lo, k_hi=hi, targets=t, seeds=(0,), name=f"gauss-{N}^3-linear{N//2}")


def config_local_ng(N: int = 256, n_bins: int = 64) -> Job:
    """Local NG at 256^3: f_NL = 5 enters as F_NL = (3/5) f_NL = 3 with the sample
    <zeta_g^2> subtracted; A=1e-2, sigma=0.5, k*=20; 64 log bins; seeds 0..3."""
    L = TWO_PI
    e, t = log_bins(N, L, n_bins)
    lo, hi = shells_from_edges(e)
    return Job(N=N, L=L, spectrum=Lognormal(1e-2, 0.5, 20.0),
               ngmap=NGMap(MAP_LOCAL, F_NL=0.6 * 5.0, G_NL=0.0),
               k_lo=lo, k_hi=hi, targets=t, seeds=(0, 1, 2, 3), name=f"localNG-fNL5-{N}^3-log{n_bins}")


def config_exptail(N: int = 512, n_bins: int = 96) -> Job:
    """Exponential-tail map at 512^3: beta=3, clip 1e-6, A=5e-3, sigma=0.3, k*=40;
    96 log bins; seeds 0..7 averaged."""
    L = TWO_PI
    e, t = log_bins(N, L, n_bins)
    lo, hi = shells_from_edges(e)
    return Job(N=N, L=L, spectrum=Lognormal(5e-3, 0.3, 40.0),
               ngmap=NGMap(MAP_EXPTAIL, beta=3.0, clip=1e-6),
               k_lo=lo, k_hi=hi, targets=t, seeds=tuple(range(8)), name=f"exptail-beta3-{N}^3-log{n_bins}")


def ensemble_params(n_real: int = 64, seed: int = 2605) -> List[dict]:
    """Per-realisation parameters of the batched ensemble: f_NL ~ U[-5, 5],
    sigma ~ U[0.2, 1.0], k* ~ U[8, 24], A = 1e-2; field seed = realisation index.
    Drawn from a NumPy PCG64 stream so both sides see the same numbers."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n_real):
        f_nl = float(rng.uniform(-5.0, 5.0))
        sigma = float(rng.uniform(0.2, 1.0))
        kstar = float(rng.uniform(8.0, 24.0))
        out.append(dict(seed=r, f_NL=f_nl, F_NL=0.6 * f_nl, sigma=sigma, k_star=kstar, A=1e-2))
    return out


def config_ensemble(N: int = 128, n_real: int = 64, n_bins: int = 32) -> List[Job]:
    L = TWO_PI
    e, t = log_bins(N, L, n_bins)
    lo, hi = shells_from_edges(e)
    jobs = []
    for p in ensemble_params(n_real):
        jobs.append(Job(N=N, L=L, spectrum=Lognormal(p["A"], p["sigma"], p["k_star"]),
                        ngmap=NGMap(MAP_LOCAL, F_NL=p["F_NL"]), k_lo=lo.copy(), k_hi=hi.copy(),
                        targets=t.copy(),
                        seeds=(p["seed"],), name=f"ens{p['seed']}-{N}^3"))
    return jobs


@dataclass
class Request:
    rid: int
    arrival: float            # seconds from stream start
    job: Job


def request_stream(n_requests: int = 3000, rate: float = 50.0, seed: int = 5050,
                   sizes=(64, 128, 256, 384), weights=(0.4, 0.3, 0.2, 0.1),
                   n_targets: int = 4) -> List[Request]:
    """Poisson arrivals (exponential gaps) of spectrum requests with a mixed
    lattice size, random log-normal parameters and a local or exponential-tail
    map (50/50).  Each request asks for n_targets thin-shell targets placed
    geometrically on [k*/2, 2 k*]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = TWO_PI
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        N = int(rng.choice(np.asarray(sizes), p=np.asarray(weights)))
        sigma = float(rng.uniform(0.2, 1.0))
        kstar = float(rng.uniform(N / 16.0, N / 6.0))
        if rng.uniform() < 0.5:
            f_nl = float(rng.uniform(-5.0, 5.0))
            m = NGMap(MAP_LOCAL, F_NL=0.6 * f_nl)
        else:
            m = NGMap(MAP_EXPTAIL, beta=float(rng.uniform(1.0, 3.0)), clip=1e-6)
        targets = kstar * np.geomspace(0.5, 2.0, n_targets)
        lo, hi = thin_shells(targets, L)
        job = Job(N=N, L=L, spectrum=Lognormal(1e-2, sigma, kstar), ngmap=m,
                  k_lo=lo, k_hi=hi, targets=targets, seeds=(int(rid),), name=f"req{rid}-{N}^3")
        out.append(Request(rid=rid, arrival=t, job=job))
    return out
