"""Gaussian realisation, non-Gaussian maps and the potential spectrum.

* Log-normal peak, Eq. (lognormal): Delta^2(k) = A/sqrt(2 pi sigma^2) exp(-ln^2(k/k*)/(2 sigma^2)).
* Dimensionful spectrum, Eq. (adimensional_P): P(k) = 2 pi^2 Delta^2(k) / k^3.
* Gaussian field: white noise w(x) (one N(0,1) per site), then
  zeta_g_hat(n) = sqrt(dV P(k_F |n|)) DFT(w)(n) with the n = 0 mode set to zero,
  and zeta_g(x) = (1/V) sum_n exp(i q.x) zeta_g_hat(n).  With this, the
  lattice two-point function is <zeta_hat zeta_hat*> = V P, the discrete form
  of the continuum definition (2 pi)^3 delta(0) P.
* Maps (Sec. VI B and the exponential-tail workload):
  local    zeta = zeta_g + F_NL (zeta_g^2 - m2) + G_NL zeta_g^3, m2 = sample mean of zeta_g^2
  exptail  zeta = -ln(max(1 - beta zeta_g, clip)) / beta
* Non-local map, Eq. (nonlocal) (Sec. VI C):
  zeta = zeta_g + (alpha_NL / k_NL^2) lap(zeta_g^2) + (beta_NL / k_NL^2) zeta_g lap(zeta_g),
  with the spectral Laplacian lap X = IDFT(-|q|^2 DFT X), q = k_F n for the
  signed index n; |q|^2 is even in every component, so the Nyquist index
  keeps its own value (reading R23).
* Potential at w = 1/3: Phi = 3(1+w)/(5+3w) zeta = 2 zeta / 3 (Sec. II), and
  Phi_hat = dV DFT(Phi).
"""
from __future__ import annotations

import math

import numpy as np

from . import lattice, rng


def lognormal_delta2(k, A, sigma, k_star):
    k = np.asarray(k, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        lk = np.log(k / k_star)
        return A / math.sqrt(2.0 * math.pi * sigma * sigma) * np.exp(-lk * lk / (2.0 * sigma * sigma))


def power_spectrum(k, A, sigma, k_star):
    k = np.asarray(k, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return 2.0 * math.pi ** 2 * lognormal_delta2(k, A, sigma, k_star) / k ** 3


def gaussian_zeta(N: int, L: float, seed: int, spectrum, noise: np.ndarray = None) -> np.ndarray:
    """Real-space Gaussian zeta_g for one seed (or for a given white noise)."""
    w = rng.white_noise(N, seed) if noise is None else noise
    what = lattice.dft_plain(w)
    n2 = lattice.n2_half(N)
    k = lattice.kf(L) * np.sqrt(n2.astype(np.float64))
    dV = (L / N) ** 3
    P = power_spectrum(k, spectrum.A, spectrum.sigma, spectrum.k_star)
    amp = np.where(n2 > 0, np.sqrt(dV * np.where(n2 > 0, P, 0.0)), 0.0)
    return lattice.inverse(amp * what, L)


def laplacian(X: np.ndarray, L: float) -> np.ndarray:
    """Spectral Laplacian of a real periodic field: IDFT(-k_F^2 |n|^2 DFT(X))."""
    N = X.shape[0]
    n2 = lattice.n2_half(N).astype(np.float64)
    return lattice.inverse(-(lattice.kf(L) ** 2) * n2 * lattice.forward(X, L), L)


def apply_map(zeta_g: np.ndarray, ngmap, L: float = None) -> np.ndarray:
    kind = ngmap.kind
    if kind == "nonlocal":
        if L is None:
            raise ValueError("the non-local map needs the box size L")
        c = 1.0 / (ngmap.k_NL * ngmap.k_NL)
        return (zeta_g + ngmap.alpha_NL * c * laplacian(zeta_g * zeta_g, L)
                + ngmap.beta_NL * c * zeta_g * laplacian(zeta_g, L))
    if kind == "gauss":
        return zeta_g.copy()
    if kind == "local":
        m2 = float(np.mean(zeta_g * zeta_g))
        return zeta_g + ngmap.F_NL * (zeta_g * zeta_g - m2) + ngmap.G_NL * zeta_g ** 3
    if kind == "exptail":
        arg = np.maximum(1.0 - ngmap.beta * zeta_g, ngmap.clip)
        return -np.log(arg) / ngmap.beta
    raise ValueError(f"unknown map {kind!r}")


def phi_hat_from_zeta(zeta: np.ndarray, L: float) -> np.ndarray:
    """Phi_hat = dV DFT(2 zeta / 3) on the half layout."""
    return lattice.forward(zeta, L) * (2.0 / 3.0)


def phi_hat(N: int, L: float, seed: int, spectrum, ngmap) -> np.ndarray:
    zg = gaussian_zeta(N, L, seed, spectrum)
    return phi_hat_from_zeta(apply_map(zg, ngmap, L), L)
